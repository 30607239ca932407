// Host side of libgmf: configuration checks, workspace planning, the seeded
// schedule of Algorithm 1 and the C ABI declared in include/gmf.h.
//
// Schedule (Algorithm 1): the row and column partitions are drawn once, from
// Fisher-Yates shuffles driven by SplitMix64 (Steele, Lea and Flood 2014) on
// sub-streams 0 and 1 of the seed; block r of the rows is the slice
// [floor(r n / R), floor((r+1) n / R)) of the row permutation (likewise for
// columns).  Step t (from 1) uses column block (t-1) mod S and row block
// floor(u_t R / 2^64), u_t being draw t-1 of sub-stream 2 (uniform, with
// replacement).  Sub-stream k starts at the (k+1)-th SplitMix64 output of the
// seed; draw j of a stream with start state x is mix(x + (j+1) * golden).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/gmf.h"
#include "gmf_kernels.hpp"

namespace {

thread_local std::string g_last_error;

int fail(int code, const std::string& msg) {
  g_last_error = msg;
  return code;
}

#define HIP_TRY(expr)                                                              \
  do {                                                                             \
    hipError_t e_ = (expr);                                                        \
    if (e_ != hipSuccess)                                                          \
      return fail(GMF_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

// ----------------------------------------------------------------- SplitMix64
constexpr uint64_t kGolden = 0x9E3779B97F4A7C15ULL;

uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}
uint64_t stream_start(uint64_t seed, uint64_t stream) { return mix64(seed + (stream + 1) * kGolden); }
uint64_t stream_draw(uint64_t start, uint64_t j) { return mix64(start + (j + 1) * kGolden); }
uint64_t below(uint64_t u, uint64_t n) {
  return (uint64_t)(((unsigned __int128)u * (unsigned __int128)n) >> 64);
}

std::vector<int> shuffle(uint64_t seed, uint64_t stream, int64_t n) {
  std::vector<int> perm(n);
  for (int64_t i = 0; i < n; ++i) perm[i] = (int)i;
  const uint64_t x0 = stream_start(seed, stream);
  for (int64_t i = n - 1; i >= 1; --i) {
    const int64_t j = (int64_t)below(stream_draw(x0, (uint64_t)(n - 1 - i)), (uint64_t)(i + 1));
    std::swap(perm[i], perm[j]);
  }
  return perm;
}

double ms_since(std::chrono::steady_clock::time_point t0) {
  return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

// ---------------------------------------------------------------- planning --
int round_up(int x, int a) { return (x + a - 1) / a * a; }
size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Rows per workgroup of the full-deviance kernel (multiple of 32).
int dev_rows_per_wg(int nr) { return std::min(256, (nr + 31) / 32 * 32); }

struct Plan {
  int64_t n = 0, m = 0;
  int R = 0, S = 0, p = 0, q = 0, d = 0, k = 0, KP = 0, KU = 0, KV = 0;
  int prec = 0, fam = 0, with_w = 0, nw = 4;
  std::vector<int> ro, co, ld, rpw, nrr, nct, nrows, mcols;
  std::vector<int64_t> coP;
  int64_t LDtot = 0;
  int rr_max = 0, ct_max = 0, nslot = 0;
  int64_t slot_u = 0, slot_v = 0, slot_dev = 0;
  int dev_tiles = 0;
  // byte offsets into the workspace
  size_t o_Yb, o_Wb, o_Prow, o_Pcol, o_Grow, o_Hrow, o_Gcol, o_Hcol, o_Upart, o_Vpart,
      o_devpart, o_devring, o_flag, o_rowperm, o_colperm, o_rowblk, o_rowloc, o_colblk,
      o_colloc, o_blkrowbase, o_blknrows, o_blkcoloff, o_blkld, o_tileblk, o_tilefirst,
      o_byoff, o_brow0, o_bcol0, o_bnb, o_bmb, o_bldy, o_brpw, o_bnct, o_devpartial,
      o_scal, o_sumsq, o_post, o_firstnz, o_ro, o_nrows, o_rpw, o_nrr, o_co, o_mcols,
      o_ld, o_nct, o_coP, o_snap, o_devpart2, o_evring, o_alphacol, o_est, o_stats, o_hopart,
      o_Yc, total;
  bool compact_room = false;   // o_Yc holds room for the 16-bit counts
  int stats_wg = 0, ho_wg = 0;
  int row_chunk = 1, col_chunk = 1, upd_sub = 1, upd_per_step = 1;
};

constexpr int kDevRing = 4096;
constexpr int kEvRing = 256;   // gmf_run evaluation results held on the device
constexpr int kDevOverlapWGs = 128;   // workgroups of the deviance that overlaps the steps
constexpr int64_t kMaxTimedSteps = 8192;
constexpr int kMaxSlots = 16;
constexpr int kTilesPerStepTarget = 256;
constexpr int kUpdPerTile = 4;   // update workgroups per tile workgroup, at most about
constexpr int kSumsqBlocks = 256;

int panel_stride_of(const gmf_config* c);

// The generic epilogue (run-time family switch, missing entries, estimated
// dispersion) serves everything but the three complete-data, fixed-dispersion
// fast paths.
bool needs_generic(const gmf_config* c) {
  return c->family > GMF_GAUSSIAN || c->allow_missing || c->estimate_phi || c->estimate_alpha;
}

std::string check_config(const gmf_config* c) {
  if (!c) return "cfg is NULL";
  if (c->n < 1 || c->m < 1) return "n and m must be >= 1";
  if (c->n > (int64_t)1 << 31 || c->m > (int64_t)1 << 31) return "n, m must be < 2^31";
  if (c->d < 1 || c->p < 0 || c->q < 0) return "need d >= 1, p >= 0, q >= 0";
  if (c->p + c->q + c->d > 64) return "p + q + d must be <= 64";
  if (c->R < 1 || c->S < 1 || c->R > c->n || c->S > c->m) return "need 1 <= R <= n, 1 <= S <= m";
  if (c->family < GMF_POISSON || c->family > GMF_INVGAUSS) return "unknown family";
  if (c->family == GMF_GAUSSIAN && c->link != GMF_LINK_IDENTITY)
    return "Gaussian family supports the identity link only";
  if (c->family == GMF_BERNOULLI && c->link != GMF_LINK_LOGIT)
    return "Bernoulli family supports the logit link only";
  if (c->family != GMF_GAUSSIAN && c->family != GMF_BERNOULLI && c->link != GMF_LINK_LOG)
    return "Poisson, NB, Gamma and inverse Gaussian families support the log link only";
  if (c->allow_missing != 0 && c->allow_missing != 1) return "allow_missing must be 0 or 1";
  if (c->estimate_phi != 0 && c->estimate_phi != 1) return "estimate_phi must be 0 or 1";
  if (c->estimate_alpha != 0 && c->estimate_alpha != 1) return "estimate_alpha must be 0 or 1";
  if (c->estimate_alpha && c->family != GMF_NEGBIN) return "estimate_alpha needs the NB family";
  if (c->estimate_phi && c->family != GMF_GAUSSIAN && c->family != GMF_GAMMA &&
      c->family != GMF_INVGAUSS)
    return "estimate_phi needs a family with a dispersion (Gaussian, Gamma, inverse Gaussian)";
  if (needs_generic(c) && c->precision != GMF_PREC_FP32)
    return "the Gamma, Bernoulli and inverse Gaussian families, missing entries and dispersion "
           "estimation run in FP32 precision";
  if (c->precision != GMF_PREC_FP32 && c->precision != GMF_PREC_BF16 &&
      c->precision != GMF_PREC_BF16X3)
    return "unknown precision";
  if (!(c->phi > 0) || !(c->nb_alpha > 0)) return "phi and nb_alpha must be > 0";
  if (!(c->rate0 > 0) || !(c->decay >= 0) || !(c->tau > 0)) return "bad learning-rate parameters";
  if (!(c->alpha1 > 0 && c->alpha1 <= 1) || !(c->alpha2 > 0 && c->alpha2 <= 1))
    return "alpha1, alpha2 must be in (0, 1]";
  if (c->bias_mode != 0 && c->bias_mode != 1) return "bias_mode must be 0 or 1";
  if (c->bias_mode == 1 && c->alpha1 >= 1.0) return "bias_mode 1 needs alpha1 < 1";
  if (!(c->damping >= 0) || !(c->eps > 0) || !std::isfinite(c->eta_max)) return "bad damping/eps/eta_max";
  for (int i = 0; i < 4; ++i)
    if (!(c->lambda[i] >= 0)) return "lambda must be >= 0";
  if (c->skip_block_deviance != 0 && c->skip_block_deviance != 1)
    return "skip_block_deviance must be 0 or 1";
  if (c->tile_rows < 0 || c->tile_rows % 32 != 0 || c->tile_rows > 4096)
    return "tile_rows must be 0 or a multiple of 32 up to 4096";
  if (c->tile_waves != 0 && c->tile_waves != 4 && c->tile_waves != 8)
    return "tile_waves must be 0, 4 or 8";
  if (c->eval_overlap != 0 && c->eval_overlap != 1) return "eval_overlap must be 0 or 1";
  if (c->tile_waves == 8 &&
      !gmf::level_supports_nw8(c->precision, panel_stride_of(c)))
    return "tile_waves = 8 needs panel stride 16 or 32 (FP32) or 32 (BF16, split BF16)";
  if (c->panel_stride != 0) {
    const int ps = c->panel_stride;
    const bool ok = (c->precision != GMF_PREC_FP32) ? (ps == 16 || ps == 32 || ps == 64)
                                                    : (ps == 16 || ps == 32 || ps == 48 || ps == 64);
    if (!ok) return "panel_stride must be 0, 16, 32, 48 or 64 (BF16, split BF16: 16, 32 or 64)";
    if (ps < c->p + c->q + c->d) return "panel_stride must be >= p + q + d";
  }
  return "";
}

// ------------------------------------------------------------- tune table --
// Rows per step tile chosen by measurement (gmf_tune) for a class of shapes:
// precision, family, panel stride and the power-of-two classes of the block
// size |I| = ceil(n/R), |J| = ceil(m/S).  Consulted when tile_rows = 0.
struct TuneKey {
  int prec, fam, KP, nb_log2, mb_log2;
  bool operator<(const TuneKey& o) const {
    if (prec != o.prec) return prec < o.prec;
    if (fam != o.fam) return fam < o.fam;
    if (KP != o.KP) return KP < o.KP;
    if (nb_log2 != o.nb_log2) return nb_log2 < o.nb_log2;
    return mb_log2 < o.mb_log2;
  }
};
struct TuneVal {
  int tile_rows;
  double us_per_step;
};
std::mutex g_tune_mu;
std::map<TuneKey, TuneVal> g_tune;

int ilog2_ceil(int64_t x) {
  int k = 0;
  while (((int64_t)1 << k) < x) ++k;
  return k;
}

int panel_stride_of(const gmf_config* c) {
  const int k = c->p + c->q + c->d;
  if (c->panel_stride > 0) return c->panel_stride;
  if (c->precision == GMF_PREC_FP32 || k <= 16) return round_up(k, 16);
  return round_up(k, 32);   // bfloat16 products of K = 32 above stride 16
}

// Wavefronts per tile workgroup: 4 unless tile_waves asks for 8.  Since the
// tile forms each entry's deviance before its contractions (fewer live
// registers), the 4-wavefront tile is the faster one at every measured shape:
// per 10000 x 1000 step at panel stride 32, FP32 58.1 against 66.2 us with 8,
// split BF16 44.0 against 52.5, BF16 34.4 against 43.8 (before its
// three-per-unit occupancy bound).
int tile_waves_for(int prec, int KP, int rpw, int tile_waves) {
  (void)rpw;
  if (tile_waves == 8 && gmf::level_supports_nw8(prec, KP)) return 8;
  return 4;
}

// Wavefronts per tile of one level launch: a launch of at most one tile per
// compute unit runs the 8-wavefront tile where it exists and the tile count
// is automatic (same products and sums in the same order as the 4-wavefront
// tile, so the results do not change): with one tile per unit the 4-wavefront
// tile leaves each SIMD one wavefront (100000 x 5000, one-step launches: BF16
// 31.6 -> 27.5 us, FP32 50.5 -> 46.3, split BF16 40.0 -> 35.0; from two
// tiles per unit on the 4-wavefront tile is faster).
int launch_waves(int nw, int tile_waves, int prec, int KP, int64_t tiles, int cu_count) {
  if (nw == 4 && tile_waves == 0 && tiles > 0 && tiles <= cu_count &&
      gmf::level_supports_nw8(prec, KP))
    return 8;
  return nw;
}

TuneKey tune_key(const gmf_config* c) {
  return TuneKey{c->precision, c->family, panel_stride_of(c),
                 ilog2_ceil((c->n + c->R - 1) / c->R), ilog2_ceil((c->m + c->S - 1) / c->S)};
}

int tune_lookup(const gmf_config* c) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  auto it = g_tune.find(tune_key(c));
  return it == g_tune.end() ? 0 : it->second.tile_rows;
}

// Update workgroups of one step: row part, column part and the
// block-deviance workgroup.
int upd_workgroups(int n_b, int m_b, int row_chunk, int col_chunk, int sub) {
  const int rw = ((n_b + row_chunk - 1) / row_chunk + sub - 1) / sub;
  const int cw = ((m_b + col_chunk - 1) / col_chunk + sub - 1) / sub;
  return rw + cw + 1;
}

void make_plan(const gmf_config* c, int with_w, Plan& P) {
  P.n = c->n; P.m = c->m; P.R = c->R; P.S = c->S;
  P.p = c->p; P.q = c->q; P.d = c->d; P.k = c->p + c->q + c->d;
  P.prec = c->precision; P.fam = needs_generic(c) ? gmf::kGeneric : c->family;
  P.with_w = with_w ? 1 : 0;
  P.KP = panel_stride_of(c);

  const int tuned_rows = c->tile_rows > 0 ? 0 : tune_lookup(c);
  P.KU = P.q + P.d; P.KV = P.p + P.d;
  P.ro.resize(P.R + 1); P.co.resize(P.S + 1);
  for (int r = 0; r <= P.R; ++r) P.ro[r] = (int)((int64_t)r * P.n / P.R);
  for (int s = 0; s <= P.S; ++s) P.co[s] = (int)((int64_t)s * P.m / P.S);
  P.ld.resize(P.S); P.coP.assign(P.S + 1, 0); P.nct.resize(P.S);
  int nct_max = 1;
  for (int s = 0; s < P.S; ++s) {
    const int ms = P.co[s + 1] - P.co[s];
    P.ld[s] = round_up(ms, 4);
    P.coP[s + 1] = P.coP[s] + P.ld[s];
    P.nct[s] = (ms + gmf::kTileCols - 1) / gmf::kTileCols;
    nct_max = std::max(nct_max, P.nct[s]);
  }
  P.LDtot = P.coP[P.S];
  P.rpw.resize(P.R); P.nrr.resize(P.R); P.nrows.resize(P.R); P.mcols.resize(P.S);
  for (int s = 0; s < P.S; ++s) P.mcols[s] = P.co[s + 1] - P.co[s];
  for (int r = 0; r < P.R; ++r) {
    const int nr = P.ro[r + 1] - P.ro[r];
    P.nrows[r] = nr;
    int rpw = round_up((int)std::ceil((double)nr * nct_max / kTilesPerStepTarget), gmf::kRowGroup);
    rpw = std::max(gmf::kRowGroup, std::min(rpw, 2048));
    if (c->tile_rows > 0) rpw = c->tile_rows;
    else if (tuned_rows > 0) rpw = tuned_rows;
    P.rpw[r] = rpw;
    P.nrr[r] = (nr + rpw - 1) / rpw;
  }
  P.rr_max = *std::max_element(P.nrr.begin(), P.nrr.end());
  P.nw = tile_waves_for(P.prec, P.KP, P.rpw[0], c->tile_waves);
  P.ct_max = nct_max;
  P.slot_u = P.slot_v = P.slot_dev = 0; P.dev_tiles = 0;
  for (int r = 0; r < P.R; ++r)
    for (int s = 0; s < P.S; ++s) {
      const int64_t nr = P.nrows[r], ms = P.mcols[s];
      P.slot_u = std::max<int64_t>(P.slot_u, (int64_t)P.nct[s] * nr * 2 * P.KU);
      P.slot_v = std::max<int64_t>(P.slot_v, (int64_t)P.nrr[r] * ms * 2 * P.KV);
      P.slot_dev = std::max<int64_t>(P.slot_dev, (int64_t)P.nrr[r] * P.nct[s]);
      P.dev_tiles += ((nr + dev_rows_per_wg((int)nr) - 1) / dev_rows_per_wg((int)nr)) * P.nct[s];
    }
  P.slot_u = (P.slot_u + 63) / 64 * 64;
  P.slot_v = (P.slot_v + 63) / 64 * 64;
  P.slot_dev = (P.slot_dev + 31) / 32 * 32;
  {
    const double slot_bytes = 4.0 * (P.slot_u + P.slot_v) + 8.0 * P.slot_dev;
    P.nslot = (int)std::max(2.0, std::min((double)kMaxSlots, (256.0 * 1024 * 1024) / slot_bytes));
  }
  const int nb = P.R * P.S;
  size_t o = 0;
  auto take = [&](size_t bytes) { size_t at = o; o = align256(o + bytes); return at; };
  P.o_Yb = take(sizeof(float) * (size_t)P.n * P.LDtot);
  P.o_Wb = take(P.with_w ? sizeof(float) * (size_t)P.n * P.LDtot : 0);
  P.compact_room = c->compact_counts != 0 && (P.fam == gmf::kPoisson || P.fam == gmf::kNegBin);
  P.o_Yc = take(P.compact_room ? sizeof(uint16_t) * (size_t)P.n * P.LDtot : 0);
  P.o_Prow = take(sizeof(float) * (size_t)P.n * P.KP);
  P.o_Pcol = take(sizeof(float) * (size_t)P.m * P.KP);
  P.o_Grow = take(sizeof(double) * (size_t)P.n * P.KU);
  P.o_Hrow = take(sizeof(double) * (size_t)P.n * P.KU);
  P.o_Gcol = take(sizeof(double) * (size_t)P.m * P.KV);
  P.o_Hcol = take(sizeof(double) * (size_t)P.m * P.KV);
  P.o_Upart = take(sizeof(float) * (size_t)P.slot_u * P.nslot);
  P.o_Vpart = take(sizeof(float) * (size_t)P.slot_v * P.nslot);
  P.o_devpart = take(sizeof(double) * (size_t)P.slot_dev * P.nslot);
  P.o_devring = take(sizeof(double) * kDevRing);
  P.o_flag = take(sizeof(int) * 4);
  P.o_rowperm = take(sizeof(int) * (size_t)P.n);
  P.o_colperm = take(sizeof(int) * (size_t)P.m);
  P.o_rowblk = take(sizeof(int) * (size_t)P.n);
  P.o_rowloc = take(sizeof(int) * (size_t)P.n);
  P.o_colblk = take(sizeof(int) * (size_t)P.m);
  P.o_colloc = take(sizeof(int) * (size_t)P.m);
  P.o_blkrowbase = take(sizeof(int64_t) * P.R);
  P.o_blknrows = take(sizeof(int) * P.R);
  P.o_blkcoloff = take(sizeof(int64_t) * P.S);
  P.o_blkld = take(sizeof(int) * P.S);
  P.o_tileblk = take(sizeof(int) * (size_t)P.dev_tiles);
  P.o_tilefirst = take(sizeof(int) * nb);
  P.o_byoff = take(sizeof(int64_t) * nb);
  P.o_brow0 = take(sizeof(int) * nb);
  P.o_bcol0 = take(sizeof(int) * nb);
  P.o_bnb = take(sizeof(int) * nb);
  P.o_bmb = take(sizeof(int) * nb);
  P.o_bldy = take(sizeof(int) * nb);
  P.o_brpw = take(sizeof(int) * nb);
  P.o_bnct = take(sizeof(int) * nb);
  P.o_devpartial = take(sizeof(double) * (size_t)P.dev_tiles);
  P.o_scal = take(sizeof(double) * 16);
  P.o_sumsq = take(sizeof(double) * kSumsqBlocks * 4);
  // gmf_run: two snapshots of both panels, two sets of deviance partials and
  // a ring of evaluation results
  P.o_snap = take(sizeof(float) * 2 * (size_t)(P.n + P.m) * P.KP);
  P.o_devpart2 = take(sizeof(double) * 2 * (size_t)P.dev_tiles);
  P.o_evring = take(sizeof(double) * 8 * kEvRing);
  P.o_post = take(sizeof(double) * gmf::postprocess_scratch_doubles(P.n, P.m, P.KP, kSumsqBlocks));
  P.o_firstnz = take(sizeof(int) * 64);
  P.o_ro = take(sizeof(int) * (P.R + 1));
  P.o_nrows = take(sizeof(int) * P.R);
  P.o_rpw = take(sizeof(int) * P.R);
  P.o_nrr = take(sizeof(int) * P.R);
  P.o_co = take(sizeof(int) * (P.S + 1));
  P.o_mcols = take(sizeof(int) * P.S);
  P.o_ld = take(sizeof(int) * P.S);
  P.o_nct = take(sizeof(int) * P.S);
  P.o_coP = take(sizeof(int64_t) * (P.S + 1));
  P.o_alphacol = take(sizeof(float) * (size_t)P.m);
  P.o_est = take(sizeof(double) * 4);
  P.stats_wg = 0;
  for (int r = 0; r < P.R; ++r) P.stats_wg = std::max(P.stats_wg, gmf::block_stats_workgroups(P.nrows[r]));
  P.o_stats = take(sizeof(double) * 3 * (size_t)P.stats_wg);
  P.ho_wg = gmf::heldout_workgroups(P.n);
  P.o_hopart = take(sizeof(double) * std::max<size_t>(8 * (size_t)P.ho_wg, 2 * (size_t)P.dev_tiles));
  P.row_chunk = std::max(1, gmf::kTileThreads / (2 * P.KU));
  P.col_chunk = std::max(1, gmf::kTileThreads / (2 * P.KV));
  // chunks per update workgroup: at most about four update workgroups per
  // step per tile workgroup (a workgroup's chunks run one after another, so
  // fewer, longer update workgroups trade start-up cost for latency)
  {
    int chunks = 1;
    for (int r = 0; r < P.R; ++r)
      for (int s = 0; s < P.S; ++s)
        chunks = std::max(chunks, (P.nrows[r] + P.row_chunk - 1) / P.row_chunk +
                                      (P.mcols[s] + P.col_chunk - 1) / P.col_chunk);
    const int per = kUpdPerTile * P.rr_max * P.ct_max;
    P.upd_sub = std::max(1, (chunks + per - 1) / per);
  }
  P.upd_per_step = 1;
  for (int r = 0; r < P.R; ++r)
    for (int s = 0; s < P.S; ++s)
      P.upd_per_step = std::max(P.upd_per_step, upd_workgroups(P.nrows[r], P.mcols[s], P.row_chunk,
                                                              P.col_chunk, P.upd_sub));
  P.total = o;
}

struct Ctx {
  gmf_config cfg;
  Plan P;
  hipStream_t st = nullptr;
  char* ws = nullptr;
  std::vector<int> row_perm, col_perm;
  uint64_t draw_start = 0;
  int64_t t = 0;
  int64_t batched_upto = 0;   // last step run by gmf_batch_run (no block deviance)
  int device = 0;             // HIP device of the context
  int cu_count = 256;         // its compute units
  bool alpha_col = false;     // a per-column NB shape was set (generic path)
  bool compact = false;       // the 16-bit counts at o_Yc are valid
  double est_init[4] = {1.0, 5.0, 0.0, 0.0};   // starting [phi, alpha] of the estimators
  std::vector<double> init_sv;   // singular values of the residual matrix (last gmf_initialize)
  int want_block_dev = 1;
  unsigned long long launches = 0;
  // optional per-task trace (caller's device buffer)
  unsigned long long* trace = nullptr;
  long long trace_cap = 0;
  unsigned long long trace_used = 0;
  // event timing of the step kernels
  bool timing = false;
  std::vector<hipEvent_t> events;   // 2 per timed launch
  int64_t timed_launches = 0;
  std::vector<unsigned char> timed_kind;   // per timed launch: 0 block-step tiles, 1 updates only
  int64_t timed_steps = 0;
  // sums of w c(y), the count-only part of half the unit deviance, per block
  // (r * S + s) and in total (float64; constant during the fit)
  std::vector<double> kblock;
  double ktotal = 0.0;
  // gmf_run: a second stream for the overlapped deviance and its events
  hipStream_t side = nullptr;
  std::vector<hipEvent_t> ev_snap, ev_done;
  hipEvent_t ev_start = nullptr;
  template <class T> T* at(size_t off) const { return reinterpret_cast<T*>(ws + off); }
};

Ctx* as_ctx(void* c) { return static_cast<Ctx*>(c); }

int row_block_of_step(const Ctx* c, int64_t t) {
  return (int)below(stream_draw(c->draw_start, (uint64_t)(t - 1)), (uint64_t)c->P.R);
}

double learning_rate(const gmf_config& c, int64_t t) {
  return c.rate0 / std::pow(1.0 + c.rate0 * c.decay * (double)t, c.tau);
}
double bias_factor(const gmf_config& c, int64_t t) {
  const double a1 = c.alpha1, a2 = c.alpha2, tt = (double)t;
  if (c.bias_mode == 0) return (1.0 - std::pow(1.0 - a2, tt)) / (1.0 - std::pow(1.0 - a1, tt));
  return (1.0 - std::pow(a2, tt)) / (1.0 - std::pow(a1, tt));
}

gmf::FamilyArgs family_args(const gmf_config& c) {
  gmf::FamilyArgs f;
  f.phi_inv = (float)(1.0 / c.phi);
  f.nb_alpha = (float)c.nb_alpha;
  f.eta_lo = (float)std::log(c.eps);
  f.eta_hi = (float)c.eta_max;
  f.code = c.family;
  f.link = c.link == GMF_LINK_IDENTITY ? gmf::kLinkIdentity
                                       : (c.link == GMF_LINK_LOGIT ? gmf::kLinkLogit : gmf::kLinkLog);
  f.alpha_col = nullptr;
  f.est = nullptr;
  return f;
}

// The family arguments of a context: with its per-column NB shape and its
// estimated dispersion / NB shape on the device when those are in use.
gmf::FamilyArgs family_args(const Ctx* c) {
  gmf::FamilyArgs f = family_args(c->cfg);
  if (c->alpha_col) f.alpha_col = c->at<float>(c->P.o_alphacol);
  if (c->cfg.estimate_phi || c->cfg.estimate_alpha) f.est = c->at<double>(c->P.o_est);
  return f;
}

int check_flag(Ctx* c) {
  int flag = 0;
  HIP_TRY(hipMemcpyAsync(&flag, c->at<int>(c->P.o_flag), sizeof(int), hipMemcpyDeviceToHost, c->st));
  HIP_TRY(hipStreamSynchronize(c->st));
  if (flag) {
    HIP_TRY(gmf::launch_fill_i32(c->at<int>(c->P.o_flag), 1, 0, c->st));
    HIP_TRY(hipStreamSynchronize(c->st));
    if (flag & 2) return fail(GMF_EINVAL, "input contains a negative, too large or non-finite value");
    if (flag & 4) return fail(GMF_ENUMERIC, "post-processing: X'X, Z'Z or a factor Gram is not positive definite");
    return fail(GMF_ENUMERIC, "a step produced a non-finite parameter");
  }
  return GMF_OK;
}

// The 16-bit counts when the context reads them (Poisson or NB on the
// fixed-shape epilogue, every count in [0, 65535]), else null.
const uint16_t* compact_counts_of(const Ctx* c) {
  const Plan& P = c->P;
  if (!c->compact || !(P.fam == gmf::kPoisson || P.fam == gmf::kNegBin)) return nullptr;
  return c->at<uint16_t>(P.o_Yc);
}

gmf::LevelArgs level_args(const Ctx* c) {
  const Plan& P = c->P;
  const gmf_config& cf = c->cfg;
  gmf::LevelArgs a;
  std::memset(&a, 0, sizeof(a));
  a.Y = c->at<float>(P.o_Yb);
  a.W = P.with_w ? c->at<float>(P.o_Wb) : nullptr;
  a.Yc = compact_counts_of(c);
  a.Prow = c->at<float>(P.o_Prow);
  a.Pcol = c->at<float>(P.o_Pcol);
  a.Grow = c->at<double>(P.o_Grow);
  a.Hrow = c->at<double>(P.o_Hrow);
  a.Gcol = c->at<double>(P.o_Gcol);
  a.Hcol = c->at<double>(P.o_Hcol);
  a.LDtot = P.LDtot;
  a.ro = c->at<int>(P.o_ro);
  a.nrows = c->at<int>(P.o_nrows);
  a.rpw = c->at<int>(P.o_rpw);
  a.nrr = c->at<int>(P.o_nrr);
  a.co = c->at<int>(P.o_co);
  a.mcols = c->at<int>(P.o_mcols);
  a.ldy = c->at<int>(P.o_ld);
  a.nct = c->at<int>(P.o_nct);
  a.coP = c->at<int64_t>(P.o_coP);
  a.rr_max = P.rr_max;
  a.ct_max = P.ct_max;
  a.n = P.n;
  a.m = P.m;
  a.Upart = c->at<float>(P.o_Upart);
  a.Vpart = c->at<float>(P.o_Vpart);
  a.devpart = c->at<double>(P.o_devpart);
  a.slot_u_elems = P.slot_u;
  a.slot_v_elems = P.slot_v;
  a.slot_dev_elems = P.slot_dev;
  a.row_chunk = P.row_chunk;
  a.col_chunk = P.col_chunk;
  a.upd_sub = P.upd_sub;
  a.upd_per_step = P.upd_per_step;
  a.f = family_args(c);
  a.fam = P.fam;
  a.p = P.p; a.q = P.q; a.d = P.d; a.KU = P.KU; a.KV = P.KV; a.KP = P.KP;
  a.lam_B = cf.lambda[0]; a.lam_A = cf.lambda[1]; a.lam_U = cf.lambda[2]; a.lam_V = cf.lambda[3];
  a.a1 = cf.alpha1; a.a2 = cf.alpha2; a.damping = cf.damping;
  a.devring = c->at<double>(P.o_devring);
  a.devring_len = kDevRing;
  a.err_flag = c->at<int>(P.o_flag);
  a.trace = c->trace;
  a.trace_cap = c->trace_cap;
  a.trace_base = 0;
  a.launch_id = 0;
  a.n_tile_steps = a.n_upd_steps = 0;
  return a;
}

// Block geometry and step size of global step t.
gmf::LevelStep make_step(const Ctx* c, int64_t t) {
  const Plan& P = c->P;
  gmf::LevelStep st;
  st.r = row_block_of_step(c, t);
  st.s = (int)((t - 1) % P.S);
  st.slot = (int)((t - 1) % P.nslot);
  st.n_b = P.nrows[st.r];
  st.m_b = P.mcols[st.s];
  st.n_rr = P.nrr[st.r];
  st.n_ct = P.nct[st.s];
  st.rpw = P.rpw[st.r];
  st.ldy = P.ld[st.s];
  st.ro = P.ro[st.r];
  st.co = P.co[st.s];
  st.pad = 0;
  st.yoff = (int64_t)P.ro[st.r] * P.LDtot + (int64_t)st.n_b * P.coP[st.s];
  st.stepsize = learning_rate(c->cfg, t) * bias_factor(c->cfg, t);
  st.t = t;
  return st;
}

// Run steps c->t+1 .. c->t+nsteps.  Step t is placed at level
// T(t) = max over its predecessors (previous step on the same row block, on the
// same column block, and on the same partial slot) of T + 2, or 0.  Launch k
// runs the tiles of level k and the updates of level k-1; oversized levels are
// split over several launches (tiles of level k never need updates of level k-1).
// With dispersion or NB-shape estimation every step depends on the one before
// it (its D1 and D2 use the estimates that step updated), so the steps run one
// after another: per step the tile launch, the block statistics at the
// pre-step parameters, the smoothed update of the estimates (weight rho_t;
// Appendix B), then the update launch.
int enqueue_steps_estimating(Ctx* c, int64_t nsteps) {
  const Plan& P = c->P;
  const bool want_dev = c->want_block_dev != 0;
  gmf::LevelArgs a = level_args(c);
  const int T = P.rr_max * P.ct_max;
  const double N = (double)P.n * (double)P.m - (double)P.m * P.p - (double)P.n * P.q -
                   (double)(P.n + P.m) * P.d - 1.0;
  for (int64_t k = 0; k < nsteps; ++k) {
    const int64_t t = c->t + 1 + k;
    const gmf::LevelStep st = make_step(c, t);
    for (int phase = 0; phase < 2; ++phase) {
      a.n_tile_steps = phase == 0 ? 1 : 0;
      a.n_upd_steps = phase == 0 ? 0 : 1;
      a.steps[0] = st;
      const int grid = phase == 0 ? T : P.upd_per_step;
      a.launch_id = c->launches++;
      a.trace_base = c->trace_used;
      c->trace_used += grid;
      hipEvent_t* ev = nullptr;
      if (c->timing && c->timed_launches < kMaxTimedSteps) {
        ev = &c->events[2 * c->timed_launches];
        c->timed_kind[c->timed_launches] = phase == 0 ? 0 : 1;
        ++c->timed_launches;
      }
      const int nw = phase == 0 ? launch_waves(P.nw, c->cfg.tile_waves, P.prec, P.KP, T, c->cu_count)
                                : P.nw;
      HIP_TRY(gmf::launch_level(P.prec, P.fam, P.KP, want_dev, nw, a, grid, c->st,
                                ev ? ev[0] : nullptr, ev ? ev[1] : nullptr));
      if (phase == 0) {
        gmf::BlockStatsArgs b{};
        b.Y = c->at<float>(P.o_Yb) + st.yoff;
        b.W = P.with_w ? c->at<float>(P.o_Wb) + st.yoff : nullptr;
        b.Prow = c->at<float>(P.o_Prow) + (int64_t)st.ro * P.KP;
        b.Pcol = c->at<float>(P.o_Pcol) + (int64_t)st.co * P.KP;
        b.ldy = st.ldy;
        b.n_b = st.n_b;
        b.m_b = st.m_b;
        b.KP = P.KP;
        b.col0 = st.co;
        b.f = family_args(c);
        b.partial = c->at<double>(P.o_stats);
        HIP_TRY(gmf::launch_block_stats(b, c->st));
        const double scale_phi = ((double)P.n * (double)P.m / ((double)st.n_b * st.m_b)) / N;
        HIP_TRY(gmf::launch_est_update(b.partial, gmf::block_stats_workgroups(st.n_b),
                                       c->at<double>(P.o_est), scale_phi,
                                       learning_rate(c->cfg, t), c->cfg.eps,
                                       c->cfg.estimate_phi, c->cfg.estimate_alpha, c->st));
      }
    }
  }
  if (c->timing) c->timed_steps += nsteps;
  c->t += nsteps;
  return GMF_OK;
}

int enqueue_steps(Ctx* c, int64_t nsteps) {
  const Plan& P = c->P;
  const bool want_dev = c->want_block_dev != 0;
  if (nsteps <= 0) return GMF_OK;
  if (c->cfg.estimate_phi || c->cfg.estimate_alpha) return enqueue_steps_estimating(c, nsteps);
  std::vector<gmf::LevelStep> steps(nsteps);
  std::vector<int> level(nsteps);
  std::vector<int> lr(P.R, -1), ls(P.S, -1), lslot(P.nslot, -1);
  int max_level = 0;
  for (int64_t k = 0; k < nsteps; ++k) {
    const int64_t t = c->t + 1 + k;
    gmf::LevelStep& st = steps[k];
    st = make_step(c, t);
    int lv = 0;
    if (lr[st.r] >= 0) lv = std::max(lv, lr[st.r] + 2);
    if (ls[st.s] >= 0) lv = std::max(lv, ls[st.s] + 2);
    if (lslot[st.slot] >= 0) lv = std::max(lv, lslot[st.slot] + 2);
    lr[st.r] = ls[st.s] = lslot[st.slot] = lv;
    level[k] = lv;
    max_level = std::max(max_level, lv);
  }
  std::vector<std::vector<int>> by_level(max_level + 1);
  for (int64_t k = 0; k < nsteps; ++k) by_level[level[k]].push_back((int)k);
  const int T = P.rr_max * P.ct_max;
  gmf::LevelArgs a = level_args(c);
  for (int lv = 0; lv <= max_level + 1; ++lv) {
    const std::vector<int> none;
    const std::vector<int>& tiles = lv <= max_level ? by_level[lv] : none;
    const std::vector<int>& upds = lv >= 1 ? by_level[lv - 1] : none;
    size_t it = 0, iu = 0;
    while (it < tiles.size() || iu < upds.size()) {
      int nt = (int)std::min<size_t>(tiles.size() - it, gmf::kMaxLevelSteps);
      int nu = (int)std::min<size_t>(upds.size() - iu, gmf::kMaxLevelSteps - nt);
      a.n_tile_steps = nt;
      a.n_upd_steps = nu;
      for (int i = 0; i < nt; ++i) a.steps[i] = steps[tiles[it + i]];
      for (int i = 0; i < nu; ++i) a.steps[nt + i] = steps[upds[iu + i]];
      it += nt;
      iu += nu;
      const int grid = nt * T + nu * P.upd_per_step;
      a.launch_id = c->launches++;
      a.trace_base = c->trace_used;
      c->trace_used += grid;
      hipEvent_t* ev = nullptr;
      if (c->timing && c->timed_launches < kMaxTimedSteps) {
        ev = &c->events[2 * c->timed_launches];
        c->timed_kind[c->timed_launches] = nt > 0 ? 0 : 1;
        ++c->timed_launches;
      }
      const int nw = launch_waves(P.nw, c->cfg.tile_waves, P.prec, P.KP, (int64_t)nt * T,
                                  c->cu_count);
      HIP_TRY(gmf::launch_level(P.prec, P.fam, P.KP, want_dev, nw, a, grid, c->st,
                                ev ? ev[0] : nullptr, ev ? ev[1] : nullptr));
    }
  }
  if (c->timing) c->timed_steps += nsteps;
  c->t += nsteps;
  return GMF_OK;
}

gmf::DevArgs dev_args(Ctx* c) {
  const Plan& P = c->P;
  gmf::DevArgs a{};
  a.Y = c->at<float>(P.o_Yb);
  a.W = P.with_w ? c->at<float>(P.o_Wb) : nullptr;
  a.Yc = compact_counts_of(c);
  a.Prow = c->at<float>(P.o_Prow);
  a.Pcol = c->at<float>(P.o_Pcol);
  a.tile_block = c->at<int>(P.o_tileblk);
  a.tile_first = c->at<int>(P.o_tilefirst);
  a.blk_yoff = c->at<int64_t>(P.o_byoff);
  a.blk_row0 = c->at<int>(P.o_brow0);
  a.blk_col0 = c->at<int>(P.o_bcol0);
  a.blk_nb = c->at<int>(P.o_bnb);
  a.blk_mb = c->at<int>(P.o_bmb);
  a.blk_ldy = c->at<int>(P.o_bldy);
  a.blk_rpw = c->at<int>(P.o_brpw);
  a.blk_nct = c->at<int>(P.o_bnct);
  a.f = family_args(c);
  a.partial = c->at<double>(P.o_devpartial);
  a.n_tiles = P.dev_tiles;
  return a;
}

// Sums of w c(y) per block from the per-tile sums of count_sum_kernel (tiles of
// a block are consecutive), in a fixed order; tileblk: tile -> block.
int count_constants(int fam, const gmf::DevArgs& da, const std::vector<int>& tileblk, int nblocks,
                    hipStream_t st, std::vector<double>& kblock, double& ktotal) {
  kblock.assign(nblocks, 0.0);
  ktotal = 0.0;
  if (fam == GMF_GAUSSIAN || da.n_tiles == 0) return GMF_OK;
  HIP_TRY(gmf::launch_count_sum(fam, da, st));
  std::vector<double> part(da.n_tiles);
  HIP_TRY(hipMemcpyAsync(part.data(), da.partial, sizeof(double) * part.size(),
                         hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  for (int t = 0; t < da.n_tiles; ++t) kblock[tileblk[t]] += part[t];
  for (double k : kblock) ktotal += k;
  return GMF_OK;
}

// Block of every full-deviance tile (the tiling of gmf_init).
std::vector<int> dev_tile_blocks(const Plan& P) {
  std::vector<int> tb;
  tb.reserve(P.dev_tiles);
  for (int r = 0; r < P.R; ++r)
    for (int s = 0; s < P.S; ++s) {
      const int nr = P.ro[r + 1] - P.ro[r];
      const int drpw = dev_rows_per_wg(nr);
      for (int k = 0; k < ((nr + drpw - 1) / drpw) * P.nct[s]; ++k) tb.push_back(r * P.S + s);
    }
  return tb;
}

// The dispersion and NB shape in use: [phi, alpha] from the device when they
// are estimated, else the configured ones.
int current_dispersion(Ctx* c, double out[2]) {
  out[0] = c->cfg.phi;
  out[1] = c->cfg.nb_alpha;
  if (c->cfg.estimate_phi || c->cfg.estimate_alpha) {
    HIP_TRY(hipMemcpyAsync(out, c->at<double>(c->P.o_est), 2 * sizeof(double),
                           hipMemcpyDeviceToHost, c->st));
    HIP_TRY(hipStreamSynchronize(c->st));
  }
  return GMF_OK;
}

int count_constants(int fam, const gmf::DevArgs& da, const std::vector<int>& tileblk, int nblocks,
                    hipStream_t st, std::vector<double>& kblock, double& ktotal);
std::vector<int> dev_tile_blocks(const Plan& P);

int compute_deviance(Ctx* c, double* total, double* pen) {
  const Plan& P = c->P;
  gmf::DevArgs a = dev_args(c);
  if (c->cfg.estimate_alpha) {   // the count-only part depends on the current shape
    const int rc = count_constants(P.fam, a, dev_tile_blocks(P), P.R * P.S, c->st, c->kblock,
                                   c->ktotal);
    if (rc != GMF_OK) return rc;
  }
  // The deviance monitor uses float32 products regardless of the step
  // precision, so its panel stride must be a float32 case (16, 32, 48, 64).
  HIP_TRY(gmf::launch_deviance(P.fam, P.KP, a, c->st));
  double* scal = c->at<double>(P.o_scal);
  double* sq = c->at<double>(P.o_sumsq);
  if (pen)
    HIP_TRY(gmf::launch_norms(c->at<float>(P.o_Prow), c->at<float>(P.o_Pcol), P.KP, P.n, P.m, P.p,
                              P.q, P.d, sq, kSumsqBlocks, c->st));
  HIP_TRY(gmf::launch_finalize(a.partial, P.dev_tiles, pen ? sq : nullptr, kSumsqBlocks,
                               c->at<int>(P.o_flag), scal, c->st));
  // one read-back: the sums and the error flag
  double h[6];
  HIP_TRY(hipMemcpyAsync(h, scal, sizeof(h), hipMemcpyDeviceToHost, c->st));
  HIP_TRY(hipStreamSynchronize(c->st));
  h[0] += 2.0 * c->ktotal;
  if (total) *total = h[0];
  if (pen) {
    const double* lam = c->cfg.lambda;
    double disp[2];
    const int rc = current_dispersion(c, disp);
    if (rc != GMF_OK) return rc;
    *pen = h[0] / (2.0 * disp[0]) +
           0.5 * (lam[0] * h[1] + lam[1] * h[2] + lam[2] * h[3] + lam[3] * h[4]);
  }
  return h[5] != 0.0 ? check_flag(c) : GMF_OK;
}

}  // namespace

// =================================================================== C ABI ==
// Resident scratch of the allocation-free projection (gmf_project_noalloc):
// one array per device, held until the process ends.  Host code never passes
// the array's name to a kernel (on the host it is only a stand-in for the
// symbol); it uses the device address from hipGetSymbolAddress, taken once per
// device with that device current (at gmf_init) and kept in scratch_addr.
constexpr size_t kScratchBytes = size_t(64) << 20;
static __device__ __align__(256) char scratch[kScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex scratch_mu;
void* scratch_addr[kMaxDevices] = {};

int resolve_scratch(int dev) {
  if (dev < 0 || dev >= kMaxDevices) return fail(GMF_EDEVICE, "device index out of range");
  std::lock_guard<std::mutex> lock(scratch_mu);
  if (scratch_addr[dev]) return GMF_OK;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !ptr)
    return fail(GMF_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
  scratch_addr[dev] = ptr;
  return GMF_OK;
}
}  // namespace

extern "C" {

void gmf_config_default(gmf_config* c) {
  if (!c) return;
  std::memset(c, 0, sizeof(*c));
  c->family = GMF_POISSON;
  c->link = GMF_LINK_LOG;
  c->precision = GMF_PREC_FP32;
  c->bias_mode = 0;
  c->d = 1;
  c->R = 10;
  c->S = 5;
  c->phi = 1.0;
  c->nb_alpha = 5.0;
  c->lambda[0] = 0.0; c->lambda[1] = 0.0; c->lambda[2] = 1.0; c->lambda[3] = 1.0;
  c->rate0 = 0.05; c->decay = 0.05; c->tau = 0.75;
  c->alpha1 = 0.1; c->alpha2 = 0.01;
  c->damping = 1e-3; c->eps = 1e-8; c->eta_max = 30.0;
  c->seed = 0;
  c->compact_counts = 1;
}

size_t gmf_workspace_bytes(const gmf_config* cfg, int32_t with_weights) {
  if (!check_config(cfg).empty()) return 0;
  Plan P;
  make_plan(cfg, with_weights, P);
  return P.total;
}

const char* gmf_last_error(void) { return g_last_error.c_str(); }

int gmf_init(void** ctx_out, const gmf_config* cfg, void* workspace, size_t ws_bytes,
             void* stream, const void* Y, int32_t y_dtype, const float* X, const float* Z,
             const float* W, const float* B0, const float* A0, const float* U0,
             const float* V0) {
  g_last_error.clear();
  if (!ctx_out) return fail(GMF_EINVAL, "ctx_out is NULL");
  *ctx_out = nullptr;
  const std::string bad = check_config(cfg);
  if (!bad.empty()) return fail(GMF_EINVAL, "invalid config: " + bad);
  if (!Y || !U0 || !V0) return fail(GMF_EINVAL, "Y, U0 and V0 must be given");
  if (y_dtype != GMF_Y_INT32 && y_dtype != GMF_Y_FLOAT32) return fail(GMF_EINVAL, "bad y_dtype");
  if (cfg->p > 0 && (!X || !B0)) return fail(GMF_EINVAL, "p > 0 needs X and B0");
  if (cfg->q > 0 && (!Z || !A0)) return fail(GMF_EINVAL, "q > 0 needs Z and A0");
  // device check: gfx950 only
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  hipDeviceProp_t prop;
  HIP_TRY(hipGetDeviceProperties(&prop, dev));
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
    return fail(GMF_EDEVICE, std::string("libgmf needs a gfx950 device, found ") + prop.gcnArchName);

  {
    const int rc = resolve_scratch(dev);
    if (rc != GMF_OK) return rc;
  }
  Ctx* c = new Ctx();
  c->cfg = *cfg;
  c->device = dev;
  c->cu_count = std::max(1, prop.multiProcessorCount);
  make_plan(cfg, W != nullptr, c->P);
  const Plan& P = c->P;
  if (!workspace || (reinterpret_cast<uintptr_t>(workspace) & 255) != 0 || ws_bytes < P.total) {
    delete c;
    return fail(GMF_EWORKSPACE, "workspace NULL, not 256-byte aligned or smaller than " +
                                    std::to_string(P.total) + " bytes");
  }
  c->ws = static_cast<char*>(workspace);
  c->want_block_dev = cfg->skip_block_deviance ? 0 : 1;
  c->st = static_cast<hipStream_t>(stream);
  c->row_perm = shuffle(cfg->seed, 0, P.n);
  c->col_perm = shuffle(cfg->seed, 1, P.m);
  c->draw_start = stream_start(cfg->seed, 2);

  // host tables
  std::vector<int> rowblk(P.n), rowloc(P.n), colblk(P.m), colloc(P.m), nrows(P.R);
  std::vector<int64_t> rowbase(P.R), coloff(P.S);
  for (int r = 0; r < P.R; ++r) {
    nrows[r] = P.ro[r + 1] - P.ro[r];
    rowbase[r] = (int64_t)P.ro[r] * P.LDtot;
    for (int i = P.ro[r]; i < P.ro[r + 1]; ++i) {
      rowblk[c->row_perm[i]] = r;
      rowloc[c->row_perm[i]] = i - P.ro[r];
    }
  }
  for (int s = 0; s < P.S; ++s) {
    coloff[s] = P.coP[s];
    for (int j = P.co[s]; j < P.co[s + 1]; ++j) {
      colblk[c->col_perm[j]] = s;
      colloc[c->col_perm[j]] = j - P.co[s];
    }
  }
  const int nb = P.R * P.S;
  std::vector<int> tileblk(P.dev_tiles), tilefirst(nb), brow0(nb), bcol0(nb), bnb(nb), bmb(nb),
      bldy(nb), brpw(nb), bnct(nb);
  // the full-deviance kernel walks kDevRows rows per workgroup (fewer, longer
  // workgroups than the step tiling); dev_tiles counts them
  std::vector<int64_t> byoff(nb);
  int tcount = 0;
  for (int r = 0; r < P.R; ++r)
    for (int s = 0; s < P.S; ++s) {
      const int b = r * P.S + s;
      const int nr = P.ro[r + 1] - P.ro[r];
      tilefirst[b] = tcount;
      byoff[b] = (int64_t)P.ro[r] * P.LDtot + (int64_t)nr * P.coP[s];
      brow0[b] = P.ro[r];
      bcol0[b] = P.co[s];
      bnb[b] = nr;
      bmb[b] = P.co[s + 1] - P.co[s];
      bldy[b] = P.ld[s];
      const int drpw = dev_rows_per_wg(nr);
      brpw[b] = drpw;
      bnct[b] = P.nct[s];
      for (int k = 0; k < ((nr + drpw - 1) / drpw) * P.nct[s]; ++k) tileblk[tcount++] = b;
    }

  hipStream_t st = c->st;
  auto h2d = [&](size_t off, const void* src, size_t bytes) {
    return hipMemcpyAsync(c->ws + off, src, bytes, hipMemcpyHostToDevice, st);
  };
  hipError_t e = hipSuccess;
#define H2D(off, vec) \
  if (e == hipSuccess) e = h2d(P.off, vec.data(), vec.size() * sizeof(vec[0]))
  H2D(o_rowperm, c->row_perm); H2D(o_colperm, c->col_perm);
  H2D(o_rowblk, rowblk); H2D(o_rowloc, rowloc); H2D(o_colblk, colblk); H2D(o_colloc, colloc);
  H2D(o_blkrowbase, rowbase); H2D(o_blknrows, nrows); H2D(o_blkcoloff, coloff);
  H2D(o_tileblk, tileblk); H2D(o_tilefirst, tilefirst); H2D(o_byoff, byoff);
  H2D(o_brow0, brow0); H2D(o_bcol0, bcol0); H2D(o_bnb, bnb); H2D(o_bmb, bmb);
  H2D(o_bldy, bldy); H2D(o_brpw, brpw); H2D(o_bnct, bnct);
#undef H2D
  if (e == hipSuccess) e = h2d(P.o_blkld, P.ld.data(), P.ld.size() * sizeof(int));
  if (e == hipSuccess) e = hipMemsetAsync(c->ws + P.o_Yb, 0, sizeof(float) * (size_t)P.n * P.LDtot, st);
  if (e == hipSuccess && P.with_w)
    e = hipMemsetAsync(c->ws + P.o_Wb, 0, sizeof(float) * (size_t)P.n * P.LDtot, st);
  if (e == hipSuccess) e = gmf::launch_fill_i32(c->at<int>(P.o_flag), 4, 0, st);
  if (e == hipSuccess)
    e = gmf::launch_permute_y(Y, y_dtype == GMF_Y_INT32, W, P.n, P.m, c->at<int>(P.o_rowblk),
                              c->at<int>(P.o_rowloc), c->at<int>(P.o_colblk),
                              c->at<int>(P.o_colloc), c->at<int64_t>(P.o_blkrowbase),
                              c->at<int>(P.o_blknrows), c->at<int64_t>(P.o_blkcoloff),
                              c->at<int>(P.o_blkld), c->at<float>(P.o_Yb),
                              P.with_w ? c->at<float>(P.o_Wb) : nullptr, c->at<int>(P.o_flag), st,
                              cfg->allow_missing, cfg->family + 1);
  // the 16-bit copy of the counts; flag[1] is set if a count does not fit
  int compact_flag = 1;
  if (e == hipSuccess && P.compact_room)
    e = gmf::launch_compact_counts(c->at<float>(P.o_Yb), (int64_t)P.n * P.LDtot,
                                   c->at<uint16_t>(P.o_Yc), c->at<int>(P.o_flag) + 1, st);
  if (e == hipSuccess && P.compact_room)
    e = hipMemcpyAsync(&compact_flag, c->at<int>(P.o_flag) + 1, sizeof(int), hipMemcpyDeviceToHost, st);
  c->est_init[0] = cfg->phi;
  c->est_init[1] = cfg->nb_alpha;
  if (e == hipSuccess) e = h2d(P.o_est, c->est_init, sizeof(c->est_init));
  if (e == hipSuccess)
    e = gmf::launch_pack_panel(X, P.p, A0, P.q, U0, P.d, c->at<int>(P.o_rowperm), P.n, P.KP,
                               c->at<float>(P.o_Prow), st);
  if (e == hipSuccess)
    e = gmf::launch_pack_panel(B0, P.p, Z, P.q, V0, P.d, c->at<int>(P.o_colperm), P.m, P.KP,
                               c->at<float>(P.o_Pcol), st);
  for (size_t off : {P.o_Grow, P.o_Hrow})
    if (e == hipSuccess) e = gmf::launch_fill_f64(c->at<double>(off), P.n * P.KU, 0.0, st);
  for (size_t off : {P.o_Gcol, P.o_Hcol})
    if (e == hipSuccess) e = gmf::launch_fill_f64(c->at<double>(off), P.m * P.KV, 0.0, st);
  if (e == hipSuccess) e = gmf::launch_fill_f64(c->at<double>(P.o_devring), kDevRing, 0.0, st);
  if (e == hipSuccess) e = h2d(P.o_ro, P.ro.data(), sizeof(int) * (P.R + 1));
  if (e == hipSuccess) e = h2d(P.o_nrows, P.nrows.data(), sizeof(int) * P.R);
  if (e == hipSuccess) e = h2d(P.o_rpw, P.rpw.data(), sizeof(int) * P.R);
  if (e == hipSuccess) e = h2d(P.o_nrr, P.nrr.data(), sizeof(int) * P.R);
  if (e == hipSuccess) e = h2d(P.o_co, P.co.data(), sizeof(int) * (P.S + 1));
  if (e == hipSuccess) e = h2d(P.o_mcols, P.mcols.data(), sizeof(int) * P.S);
  if (e == hipSuccess) e = h2d(P.o_ld, P.ld.data(), sizeof(int) * P.S);
  if (e == hipSuccess) e = h2d(P.o_nct, P.nct.data(), sizeof(int) * P.S);
  if (e == hipSuccess) e = h2d(P.o_coP, P.coP.data(), sizeof(int64_t) * (P.S + 1));
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) {
    delete c;
    return fail(GMF_EDEVICE, std::string("gmf_init: ") + hipGetErrorString(e));
  }
  c->compact = P.compact_room && compact_flag == 0;
  int rc = check_flag(c);
  if (rc == GMF_OK)
    rc = count_constants(P.fam, dev_args(c), tileblk, nb, st, c->kblock, c->ktotal);
  if (rc != GMF_OK) {
    delete c;
    return rc;
  }
  *ctx_out = c;
  return GMF_OK;
}

int gmf_compact_counts(void* ctx) {
  if (!ctx) return fail(GMF_EINVAL, "ctx is NULL");
  return compact_counts_of(as_ctx(ctx)) != nullptr ? 1 : 0;
}

int gmf_set_precision(void* ctx, int32_t precision) {
  if (!ctx) return fail(GMF_EINVAL, "ctx is NULL");
  Ctx* c = as_ctx(ctx);
  Plan& P = c->P;
  if (precision != GMF_PREC_FP32 && precision != GMF_PREC_BF16 && precision != GMF_PREC_BF16X3)
    return fail(GMF_EINVAL, "unknown precision");
  if (P.fam == gmf::kGeneric && precision != GMF_PREC_FP32)
    return fail(GMF_EINVAL, "this context runs the generic FP32 epilogue (family, missing entries, "
                            "per-column NB shape or dispersion estimation)");
  const bool ok = (precision != GMF_PREC_FP32) ? (P.KP == 16 || P.KP == 32 || P.KP == 64) : true;
  if (!ok) return fail(GMF_EINVAL, "BF16 needs panel stride 16, 32 or 64 (set panel_stride at init)");
  const int tw = c->cfg.tile_waves;
  if (tw == 8 && !gmf::level_supports_nw8(precision, P.KP))
    return fail(GMF_EINVAL, "tile_waves = 8 is not available for this precision and panel stride");
  P.prec = precision;
  c->cfg.precision = precision;
  P.nw = tile_waves_for(P.prec, P.KP, P.rpw[0], tw);
  return GMF_OK;
}

int gmf_step(void* ctx, int64_t nsteps) {
  if (!ctx) return fail(GMF_EINVAL, "ctx is NULL");
  if (nsteps < 0) return fail(GMF_EINVAL, "nsteps < 0");
  return enqueue_steps(as_ctx(ctx), nsteps);
}

int gmf_deviance(void* ctx, double* total_host, double* penalized_host) {
  if (!ctx) return fail(GMF_EINVAL, "ctx is NULL");
  return compute_deviance(as_ctx(ctx), total_host, penalized_host);
}

int gmf_row_deviance(void* ctx, double* per_row) {
  if (!ctx) return fail(GMF_EINVAL, "ctx is NULL");
  if (!per_row) return fail(GMF_EINVAL, "per_row is NULL");
  Ctx* c = as_ctx(ctx);
  const Plan& P = c->P;
  gmf::RowDevArgs a{};
  a.Yb = c->at<float>(P.o_Yb);
  a.Wb = P.with_w ? c->at<float>(P.o_Wb) : nullptr;
  a.Prow = c->at<float>(P.o_Prow);
  a.Pcol = c->at<float>(P.o_Pcol);
  a.rowblk = c->at<int>(P.o_rowblk);
  a.rowloc = c->at<int>(P.o_rowloc);
  a.ro = c->at<int>(P.o_ro);
  a.nrows = c->at<int>(P.o_nrows);
  a.rowbase = c->at<int64_t>(P.o_blkrowbase);
  a.co = c->at<int>(P.o_co);
  a.mcols = c->at<int>(P.o_mcols);
  a.coloff = c->at<int64_t>(P.o_blkcoloff);
  a.ld = c->at<int>(P.o_ld);
  a.n = P.n;
  a.S = P.S;
  a.f = family_args(c);
  a.out = per_row;
  HIP_TRY(gmf::launch_row_deviance(P.fam, P.KP, a, c->st));
  return GMF_OK;
}

int gmf_fit(void* ctx, int32_t max_epochs, double tol, int32_t eval_every,
            double* dev_trace_host, int32_t* epochs_done_host) {
  if (!ctx) return fail(GMF_EINVAL, "ctx is NULL");
  if (max_epochs < 0 || eval_every < 1) return fail(GMF_EINVAL, "bad max_epochs / eval_every");
  Ctx* c = as_ctx(ctx);
  const int64_t per_epoch = (int64_t)c->P.R * c->P.S;
  double prev = NAN;
  int ntrace = 0;
  int done = 0;
  bool conv = false;
  for (int e = 1; e <= max_epochs; ++e) {
    int rc = enqueue_steps(c, per_epoch);
    if (rc != GMF_OK) return rc;
    done = e;
    if (e % eval_every == 0) {
      double dev = 0;
      rc = compute_deviance(c, &dev, nullptr);
      if (rc != GMF_OK) {
        if (epochs_done_host) *epochs_done_host = done;
        return rc;
      }
      if (dev_trace_host) dev_trace_host[ntrace] = dev;
      ++ntrace;
      if (tol > 0 && std::isfinite(prev) && std::fabs(prev - dev) <= tol * std::fabs(dev)) {
        conv = true;
        break;
      }
      prev = dev;
    }
  }
  if (epochs_done_host) *epochs_done_host = done;
  const int rc = check_flag(c);
  if (rc != GMF_OK) return rc;
  if (tol > 0 && !conv) return fail(GMF_ENOTCONV, "tolerance not met within max_epochs");
  return GMF_OK;
}

int gmf_block_deviance(void* ctx, double* out_host, int64_t count) {
  if (!ctx || !out_host) return fail(GMF_EINVAL, "NULL argument");
  Ctx* c = as_ctx(ctx);
  if (count < 0 || count > c->t || count > kDevRing) return fail(GMF_EINVAL, "bad count");
  if (!c->want_block_dev) return fail(GMF_EINVAL, "block deviance is off (skip_block_deviance)");
  if (c->cfg.estimate_alpha)
    return fail(GMF_EINVAL, "block deviances are not kept while the NB shape is estimated "
                            "(their count-only part changes with it); use gmf_deviance");
  if (count > 0 && c->t - count + 1 <= c->batched_upto)
    return fail(GMF_EINVAL, "the requested steps include steps run by gmf_batch_run, which "
                            "form no block deviance");
  std::vector<double> ring(kDevRing);
  HIP_TRY(hipMemcpyAsync(ring.data(), c->at<double>(c->P.o_devring), sizeof(double) * kDevRing,
                         hipMemcpyDeviceToHost, c->st));
  HIP_TRY(hipStreamSynchronize(c->st));
  for (int64_t k = 0; k < count; ++k) {
    const int64_t t = c->t - count + 1 + k;
    const int r = row_block_of_step(c, t), s = (int)((t - 1) % c->P.S);
    out_host[k] = ring[(t - 1) % kDevRing] + 2.0 * c->kblock[r * c->P.S + s];
  }
  return check_flag(c);
}

int gmf_get_params(void* ctx, float* B, float* A, float* U, float* V, int32_t postprocess) {
  if (!ctx) return fail(GMF_EINVAL, "ctx is NULL");
  Ctx* c = as_ctx(ctx);
  const Plan& P = c->P;
  if (postprocess) {
    gmf::PostArgs a;
    a.Prow = c->at<float>(P.o_Prow);
    a.Pcol = c->at<float>(P.o_Pcol);
    a.n = P.n; a.m = P.m; a.p = P.p; a.q = P.q; a.d = P.d; a.KP = P.KP;
    a.row_perm = c->at<int>(P.o_rowperm);
    a.col_perm = c->at<int>(P.o_colperm);
    a.gram_part = c->at<double>(P.o_post);
    a.small = nullptr;
    a.first_nz = c->at<int>(P.o_firstnz);
    a.err_flag = c->at<int>(P.o_flag);
    a.B = B; a.A = A; a.U = U; a.V = V;
    a.nblocks_row = kSumsqBlocks;
    a.nblocks_col = kSumsqBlocks;
    HIP_TRY(gmf::launch_postprocess(a, c->st));
    return check_flag(c);
  }
  const int* rp = c->at<int>(P.o_rowperm);
  const int* cp = c->at<int>(P.o_colperm);
  HIP_TRY(gmf::launch_unpack_panel(c->at<float>(P.o_Pcol), P.KP, cp, P.m, 0, P.p, B, c->st));
  HIP_TRY(gmf::launch_unpack_panel(c->at<float>(P.o_Prow), P.KP, rp, P.n, P.p, P.q, A, c->st));
  HIP_TRY(gmf::launch_unpack_panel(c->at<float>(P.o_Prow), P.KP, rp, P.n, P.p + P.q, P.d, U, c->st));
  HIP_TRY(gmf::launch_unpack_panel(c->at<float>(P.o_Pcol), P.KP, cp, P.m, P.p + P.q, P.d, V, c->st));
  return check_flag(c);
}

int gmf_set_params(void* ctx, const float* B, const float* A, const float* U, const float* V) {
  if (!ctx) return fail(GMF_EINVAL, "ctx is NULL");
  Ctx* c = as_ctx(ctx);
  const Plan& P = c->P;
  if (!U || !V || (P.p > 0 && !B) || (P.q > 0 && !A)) return fail(GMF_EINVAL, "missing array");
  // The covariates are kept: read them back out of the panels first.
  // Packing rewrites whole rows, so stage X and Z through the panel itself:
  // pack only the parameter columns by unpacking X/Z into scratch.
  float* stage = reinterpret_cast<float*>(c->at<double>(P.o_post));
  const size_t need = (size_t)std::max<int64_t>(P.n * P.p, P.m * P.q);
  if (need * sizeof(float) > sizeof(double) * gmf::postprocess_scratch_doubles(P.n, P.m, P.KP, kSumsqBlocks))
    return fail(GMF_EINVAL, "internal: scratch too small");
  const int* rp = c->at<int>(P.o_rowperm);
  const int* cp = c->at<int>(P.o_colperm);
  if (P.p > 0) HIP_TRY(gmf::launch_unpack_panel(c->at<float>(P.o_Prow), P.KP, rp, P.n, 0, P.p, stage, c->st));
  HIP_TRY(gmf::launch_pack_panel(stage, P.p, A, P.q, U, P.d, rp, P.n, P.KP, c->at<float>(P.o_Prow), c->st));
  if (P.q > 0) HIP_TRY(gmf::launch_unpack_panel(c->at<float>(P.o_Pcol), P.KP, cp, P.m, P.p, P.q, stage, c->st));
  HIP_TRY(gmf::launch_pack_panel(B, P.p, stage, P.q, V, P.d, cp, P.m, P.KP, c->at<float>(P.o_Pcol), c->st));
  return check_flag(c);
}

int gmf_get_moments(void* ctx, double* Grow, double* Hrow, double* Gcol, double* Hcol) {
  if (!ctx) return fail(GMF_EINVAL, "ctx is NULL");
  Ctx* c = as_ctx(ctx);
  const Plan& P = c->P;
  const int* rp = c->at<int>(P.o_rowperm);
  const int* cp = c->at<int>(P.o_colperm);
  HIP_TRY(gmf::launch_unpack_moments(c->at<double>(P.o_Grow), P.KU, rp, P.n, Grow, c->st));
  HIP_TRY(gmf::launch_unpack_moments(c->at<double>(P.o_Hrow), P.KU, rp, P.n, Hrow, c->st));
  HIP_TRY(gmf::launch_unpack_moments(c->at<double>(P.o_Gcol), P.KV, cp, P.m, Gcol, c->st));
  HIP_TRY(gmf::launch_unpack_moments(c->at<double>(P.o_Hcol), P.KV, cp, P.m, Hcol, c->st));
  return check_flag(c);
}

int gmf_get_schedule(void* ctx, int32_t* row_perm_host, int32_t* col_perm_host,
                     int64_t t_first, int64_t count, int32_t* r_host) {
  if (!ctx) return fail(GMF_EINVAL, "ctx is NULL");
  Ctx* c = as_ctx(ctx);
  if (row_perm_host) std::memcpy(row_perm_host, c->row_perm.data(), sizeof(int) * c->P.n);
  if (col_perm_host) std::memcpy(col_perm_host, c->col_perm.data(), sizeof(int) * c->P.m);
  if (r_host) {
    if (t_first < 1 || count < 0) return fail(GMF_EINVAL, "t_first must be >= 1, count >= 0");
    for (int64_t k = 0; k < count; ++k) r_host[k] = row_block_of_step(c, t_first + k);
  }
  return GMF_OK;
}

int gmf_schedule_host(uint64_t seed, int64_t n, int64_t m, int32_t R, int64_t t_first,
                      int64_t count, int32_t* row_perm_host, int32_t* col_perm_host,
                      int32_t* r_host) {
  if (n < 0 || m < 0 || R < 1 || count < 0 || (r_host && t_first < 1))
    return fail(GMF_EINVAL, "bad schedule arguments");
  if (row_perm_host) {
    const std::vector<int> rp = shuffle(seed, 0, n);
    std::memcpy(row_perm_host, rp.data(), sizeof(int) * n);
  }
  if (col_perm_host) {
    const std::vector<int> cp = shuffle(seed, 1, m);
    std::memcpy(col_perm_host, cp.data(), sizeof(int) * m);
  }
  if (r_host) {
    const uint64_t x0 = stream_start(seed, 2);
    for (int64_t k = 0; k < count; ++k)
      r_host[k] = (int)below(stream_draw(x0, (uint64_t)(t_first + k - 1)), (uint64_t)R);
  }
  return GMF_OK;
}

int64_t gmf_steps_done(void* ctx) { return ctx ? as_ctx(ctx)->t : -1; }

int gmf_sync(void* ctx) {
  if (!ctx) return fail(GMF_EINVAL, "ctx is NULL");
  return check_flag(as_ctx(ctx));
}



// ------------------------------------------------------------ rank selection --
// Section 4.2: spectral thresholding on the residual matrix of the
// initialization, read by the eigenvalue-gap ("edge distribution") estimator
// of Onatski (2010); and the out-of-sample criterion, the rank whose fits
// have the smallest mean held-out deviance over the folds.
extern "C" int gmf_init_spectrum(void* ctx, double* sv_host, int32_t count) {
  if (!ctx || !sv_host) return fail(GMF_EINVAL, "NULL argument");
  Ctx* c = as_ctx(ctx);
  if (c->init_sv.empty()) return fail(GMF_EINVAL, "no initialization has run on this context");
  if (count < 1 || count > (int32_t)c->init_sv.size())
    return fail(GMF_EINVAL, "count must be in [1, k of the last initialization]");
  for (int j = 0; j < count; ++j) sv_host[j] = c->init_sv[j];
  return GMF_OK;
}

extern "C" int gmf_rank_eigengap(const double* eigenvalues, int32_t count, int32_t rmax,
                                 int32_t* rank_host) {
  if (!eigenvalues || !rank_host) return fail(GMF_EINVAL, "NULL argument");
  if (rmax < 1 || count < rmax + 5) return fail(GMF_EINVAL, "need rmax >= 1 and count >= rmax + 5");
  for (int i = 0; i + 1 < count; ++i)
    if (!(eigenvalues[i] >= eigenvalues[i + 1]) || !std::isfinite(eigenvalues[i]))
      return fail(GMF_EINVAL, "eigenvalues must be finite and sorted in descending order");
  int j = rmax + 1, r = 0, r_prev = -1;
  for (int it = 0; it < 100; ++it) {
    // least-squares slope of lambda_j .. lambda_{j+4} on (j-1)^{2/3} .. (j+3)^{2/3}
    double xs[5], ys[5], mx = 0.0, my = 0.0;
    for (int q = 0; q < 5; ++q) {
      xs[q] = std::pow((double)(j + q - 1), 2.0 / 3.0);
      ys[q] = eigenvalues[j + q - 1];
      mx += xs[q] / 5.0;
      my += ys[q] / 5.0;
    }
    double sxy = 0.0, sxx = 0.0;
    for (int q = 0; q < 5; ++q) {
      sxy += (xs[q] - mx) * (ys[q] - my);
      sxx += (xs[q] - mx) * (xs[q] - mx);
    }
    const double delta = 2.0 * std::fabs(sxy / sxx);
    r = 0;
    for (int i = 1; i <= rmax; ++i)
      if (eigenvalues[i - 1] - eigenvalues[i] >= delta) r = i;
    if (r == r_prev) break;
    r_prev = r;
    j = r + 1;
  }
  *rank_host = r;
  return GMF_OK;
}

extern "C" int gmf_rank_select_cv(const double* dev_host, int32_t nranks, int32_t nfolds,
                                  int32_t* best_host) {
  if (!dev_host || !best_host || nranks < 1 || nfolds < 1) return fail(GMF_EINVAL, "bad arguments");
  int best = -1;
  double best_mean = 0.0;
  for (int r = 0; r < nranks; ++r) {
    double s = 0.0;
    for (int f = 0; f < nfolds; ++f) s += dev_host[(size_t)r * nfolds + f];
    const double mean = s / nfolds;
    if (!std::isfinite(mean)) return fail(GMF_EINVAL, "non-finite held-out deviance");
    if (best < 0 || mean < best_mean) {
      best = r;
      best_mean = mean;
    }
  }
  *best_host = best;
  return GMF_OK;
}

// ------------------------------------------------------------ projection --
namespace {

struct ProjPlan {
  int64_t n_new = 0;
  int dev_rpw = 0, dev_tiles = 0;
  size_t o_Yb, o_Prow, o_Pcol, o_Grow, o_Hrow, o_iota, o_zero, o_rowbase,
      o_nrows, o_tileblk, o_tilefirst, o_byoff, o_brow0, o_bcol0, o_bnb, o_bmb, o_bldy, o_brpw,
      o_bnct, o_devpartial, o_scal, o_tmpB, o_tmpZ, o_tmpV, o_count, o_pcolorig, o_Yc, o_cflag,
      total;
  bool compact_room = false;   // room for the new rows' 16-bit counts
};

bool make_proj_plan(const Ctx* c, int64_t n_new, ProjPlan& Q) {
  const Plan& P = c->P;
  if (n_new < 1 || n_new > ((int64_t)1 << 31) - 1) return false;
  Q.n_new = n_new;
  Q.dev_rpw = dev_rows_per_wg((int)std::min<int64_t>(n_new, 1 << 30));
  Q.dev_tiles = 0;
  for (int s = 0; s < P.S; ++s) Q.dev_tiles += (int)((n_new + Q.dev_rpw - 1) / Q.dev_rpw) * P.nct[s];
  size_t o = 0;
  auto take = [&](size_t bytes) { size_t at = o; o = align256(o + bytes); return at; };
  Q.o_Yb = take(sizeof(float) * (size_t)n_new * P.LDtot);
  Q.o_Prow = take(sizeof(float) * (size_t)n_new * P.KP);
  Q.o_Pcol = take(sizeof(float) * (size_t)P.m * P.KP);
  Q.o_Grow = take(sizeof(double) * (size_t)n_new * P.KU);
  Q.o_Hrow = take(sizeof(double) * (size_t)n_new * P.KU);
  Q.o_iota = take(sizeof(int) * (size_t)n_new);
  Q.o_zero = take(sizeof(int) * (size_t)n_new);
  Q.o_rowbase = take(sizeof(int64_t));
  Q.o_nrows = take(sizeof(int));
  Q.o_tileblk = take(sizeof(int) * (size_t)Q.dev_tiles);
  Q.o_tilefirst = take(sizeof(int) * P.S);
  Q.o_byoff = take(sizeof(int64_t) * P.S);
  Q.o_brow0 = take(sizeof(int) * P.S);
  Q.o_bcol0 = take(sizeof(int) * P.S);
  Q.o_bnb = take(sizeof(int) * P.S);
  Q.o_bmb = take(sizeof(int) * P.S);
  Q.o_bldy = take(sizeof(int) * P.S);
  Q.o_brpw = take(sizeof(int) * P.S);
  Q.o_bnct = take(sizeof(int) * P.S);
  Q.o_devpartial = take(sizeof(double) * (size_t)Q.dev_tiles);
  Q.o_scal = take(sizeof(double) * 16);
  Q.o_tmpB = take(sizeof(float) * (size_t)P.m * std::max(P.p, 1));
  Q.o_tmpZ = take(sizeof(float) * (size_t)P.m * std::max(P.q, 1));
  Q.o_tmpV = take(sizeof(float) * (size_t)P.m * P.d);
  Q.o_count = take(sizeof(unsigned long long) * 2);
  Q.o_pcolorig = take(sizeof(float) * (size_t)P.m * P.KP);
  Q.compact_room = P.compact_room;
  Q.o_Yc = take(Q.compact_room ? sizeof(uint16_t) * (size_t)n_new * P.LDtot : 0);
  Q.o_cflag = take(sizeof(int));
  Q.total = o;
  return true;
}

}  // namespace

extern "C" size_t gmf_project_workspace_bytes(void* ctx, int64_t n_new) {
  if (!ctx) return 0;
  ProjPlan Q;
  if (!make_proj_plan(as_ctx(ctx), n_new, Q)) return 0;
  return Q.total;
}

namespace {

// Starting values of the projected rows: the caller's (A0, U0), or built on
// the device (row intercept, then the candidate scores or 0 per row).
enum ProjInit { kInitGiven = 0, kInitWarm = 1 };

int project_impl(Ctx* c, void* ws, size_t ws_bytes, const void* Ynew, int32_t y_dtype,
                 int64_t n_new, const float* Xnew, const float* A0, const float* U0,
                 int init_mode, const float* Ucand, int32_t epochs, int32_t frozen,
                 float* A_out, float* U_out, double* dev_trace_host, double* epoch_ms_host,
                 int64_t* fallback_host) {
  const auto t_start = std::chrono::steady_clock::now();
  const Plan& P = c->P;
  if (P.fam == gmf::kGeneric)
    return fail(GMF_EINVAL, "projection runs the Poisson, NB and Gaussian complete-data paths only");
  ProjPlan Q;
  if (!make_proj_plan(c, n_new, Q)) return fail(GMF_EINVAL, "bad n_new");
  if (!Ynew || !U_out || (P.p > 0 && !Xnew) || (P.q > 0 && !A_out))
    return fail(GMF_EINVAL, "missing array");
  if (init_mode == kInitGiven && (!U0 || (P.q > 0 && !A0)))
    return fail(GMF_EINVAL, "missing starting values");
  if (epoch_ms_host && !dev_trace_host)
    return fail(GMF_EINVAL, "epoch_ms_host needs dev_trace_host");
  if (y_dtype != GMF_Y_INT32 && y_dtype != GMF_Y_FLOAT32) return fail(GMF_EINVAL, "bad y_dtype");
  if (epochs < 0) return fail(GMF_EINVAL, "epochs < 0");
  if (!ws || (reinterpret_cast<uintptr_t>(ws) & 255) != 0 || ws_bytes < Q.total)
    return fail(GMF_EWORKSPACE, "projection workspace NULL, misaligned or smaller than " +
                                    std::to_string(Q.total) + " bytes");
  char* W = static_cast<char*>(ws);
  auto at = [&](size_t off) { return W + off; };
  hipStream_t st = c->st;
  // ---- tables: one row block (all new rows), the context's column blocks
  HIP_TRY(gmf::launch_iota(reinterpret_cast<int*>(at(Q.o_iota)), n_new, st));
  HIP_TRY(gmf::launch_fill_i32(reinterpret_cast<int*>(at(Q.o_zero)), n_new, 0, st));
  const int64_t rowbase = 0;
  const int nrows = (int)n_new;
  HIP_TRY(hipMemcpyAsync(at(Q.o_rowbase), &rowbase, sizeof(rowbase), hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(at(Q.o_nrows), &nrows, sizeof(nrows), hipMemcpyHostToDevice, st));
  std::vector<int> tileblk(Q.dev_tiles), tilefirst(P.S), brow0(P.S, 0), bcol0(P.S), bnb(P.S), bmb(P.S),
      bldy(P.S), brpw(P.S, Q.dev_rpw), bnct(P.S);
  std::vector<int64_t> byoff(P.S);
  int tc = 0;
  for (int s = 0; s < P.S; ++s) {
    tilefirst[s] = tc;
    byoff[s] = (int64_t)n_new * P.coP[s];
    bcol0[s] = P.co[s];
    bnb[s] = (int)n_new;
    bmb[s] = P.mcols[s];
    bldy[s] = P.ld[s];
    bnct[s] = P.nct[s];
    const int tiles = (int)((n_new + Q.dev_rpw - 1) / Q.dev_rpw) * P.nct[s];
    for (int k = 0; k < tiles; ++k) tileblk[tc++] = s;
  }
  HIP_TRY(hipMemcpyAsync(at(Q.o_tileblk), tileblk.data(), sizeof(int) * tileblk.size(), hipMemcpyHostToDevice, st));
#define PH2D(off, vec) HIP_TRY(hipMemcpyAsync(at(Q.off), vec.data(), sizeof(vec[0]) * vec.size(), hipMemcpyHostToDevice, st))
  PH2D(o_tilefirst, tilefirst); PH2D(o_byoff, byoff); PH2D(o_brow0, brow0); PH2D(o_bcol0, bcol0);
  PH2D(o_bnb, bnb); PH2D(o_bmb, bmb); PH2D(o_bldy, bldy); PH2D(o_brpw, brpw); PH2D(o_bnct, bnct);
#undef PH2D
  // ---- data: Y in column-block-major order, the new row panel, the frozen column panel
  float* Yb = reinterpret_cast<float*>(at(Q.o_Yb));
  HIP_TRY(gmf::launch_fill_i32(reinterpret_cast<int*>(Yb), n_new * P.LDtot, 0, st));
  HIP_TRY(gmf::launch_permute_y(Ynew, y_dtype == GMF_Y_INT32, nullptr, n_new, P.m,
                                reinterpret_cast<int*>(at(Q.o_zero)), reinterpret_cast<int*>(at(Q.o_iota)),
                                c->at<int>(P.o_colblk), c->at<int>(P.o_colloc),
                                reinterpret_cast<int64_t*>(at(Q.o_rowbase)), reinterpret_cast<int*>(at(Q.o_nrows)),
                                c->at<int64_t>(P.o_blkcoloff), c->at<int>(P.o_blkld), Yb, nullptr,
                                c->at<int>(P.o_flag), st));
  // the 16-bit copy of the new counts, used when every count fits
  const uint16_t* Yc = nullptr;
  if (Q.compact_room) {
    int* cflag = reinterpret_cast<int*>(at(Q.o_cflag));
    uint16_t* Ycw = reinterpret_cast<uint16_t*>(at(Q.o_Yc));
    HIP_TRY(gmf::launch_fill_i32(cflag, 1, 0, st));
    HIP_TRY(gmf::launch_compact_counts(Yb, n_new * P.LDtot, Ycw, cflag, st));
    int h = 1;
    HIP_TRY(hipMemcpyAsync(&h, cflag, sizeof(int), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    if (h == 0) Yc = Ycw;
  }
  float* Prow = reinterpret_cast<float*>(at(Q.o_Prow));
  if (init_mode == kInitGiven)
    HIP_TRY(gmf::launch_pack_panel(Xnew, P.p, A0, P.q, U0, P.d, reinterpret_cast<int*>(at(Q.o_iota)),
                                   n_new, P.KP, Prow, st));
  else   // X only; Gamma and U are filled below
    HIP_TRY(gmf::launch_pack_panel(Xnew, P.p, nullptr, 0, nullptr, 0, reinterpret_cast<int*>(at(Q.o_iota)),
                                   n_new, P.KP, Prow, st));
  float* Pcol = reinterpret_cast<float*>(at(Q.o_Pcol));
  if (frozen) {
    float* tB = reinterpret_cast<float*>(at(Q.o_tmpB));
    float* tZ = reinterpret_cast<float*>(at(Q.o_tmpZ));
    float* tV = reinterpret_cast<float*>(at(Q.o_tmpV));
    gmf::PostArgs pa;
    pa.Prow = c->at<float>(P.o_Prow);
    pa.Pcol = c->at<float>(P.o_Pcol);
    pa.n = P.n; pa.m = P.m; pa.p = P.p; pa.q = P.q; pa.d = P.d; pa.KP = P.KP;
    pa.row_perm = c->at<int>(P.o_rowperm);
    pa.col_perm = c->at<int>(P.o_colperm);
    pa.gram_part = c->at<double>(P.o_post);
    pa.small = nullptr;
    pa.first_nz = c->at<int>(P.o_firstnz);
    pa.err_flag = c->at<int>(P.o_flag);
    pa.B = P.p > 0 ? tB : nullptr; pa.A = nullptr; pa.U = nullptr; pa.V = tV;
    pa.nblocks_row = kSumsqBlocks; pa.nblocks_col = kSumsqBlocks;
    HIP_TRY(gmf::launch_postprocess(pa, st));
    HIP_TRY(gmf::launch_unpack_panel(c->at<float>(P.o_Pcol), P.KP, c->at<int>(P.o_colperm), P.m, P.p, P.q, tZ, st));
    HIP_TRY(gmf::launch_pack_panel(tB, P.p, tZ, P.q, tV, P.d, c->at<int>(P.o_colperm), P.m, P.KP, Pcol, st));
  } else {
    HIP_TRY(hipMemcpyAsync(Pcol, c->at<float>(P.o_Pcol), sizeof(float) * (size_t)P.m * P.KP,
                           hipMemcpyDeviceToDevice, st));
  }
  if (init_mode == kInitWarm) {
    gmf::WarmArgs wa;
    wa.Y = Ynew; wa.n = n_new; wa.m = (int)P.m; wa.p = P.p; wa.q = P.q; wa.d = P.d; wa.KP = P.KP;
    // the frozen column panel in the caller's column order
    float* Pco = reinterpret_cast<float*>(at(Q.o_pcolorig));
    HIP_TRY(gmf::launch_unpack_panel(Pcol, P.KP, c->at<int>(P.o_colperm), P.m, 0, P.KP, Pco, st));
    wa.Prow = Prow; wa.Pcol_orig = Pco;
    wa.f = family_args(c->cfg);
    wa.Ucand = Ucand; wa.dev_out = nullptr;
    wa.fallback = reinterpret_cast<unsigned long long*>(at(Q.o_count));
    const bool y_int = y_dtype == GMF_Y_INT32;
    HIP_TRY(gmf::launch_row_intercept(wa, y_int, P.fam != GMF_GAUSSIAN, st));
    if (Ucand) {
      HIP_TRY(gmf::launch_fill_f64(reinterpret_cast<double*>(at(Q.o_count)), 1, 0.0, st));
      HIP_TRY(gmf::launch_row_select(wa, P.fam, y_int, st));
      if (fallback_host) {
        unsigned long long cnt = 0;
        HIP_TRY(hipMemcpyAsync(&cnt, at(Q.o_count), sizeof(cnt), hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        *fallback_host = (int64_t)cnt;
      }
    } else if (fallback_host) {
      *fallback_host = 0;
    }
  }
  double* Grow = reinterpret_cast<double*>(at(Q.o_Grow));
  double* Hrow = reinterpret_cast<double*>(at(Q.o_Hrow));
  HIP_TRY(gmf::launch_fill_f64(Grow, n_new * P.KU, 0.0, st));
  HIP_TRY(gmf::launch_fill_f64(Hrow, n_new * P.KU, 0.0, st));

  // ---- deviance of the new rows
  gmf::DevArgs da{};
  da.Y = Yb; da.W = nullptr; da.Yc = Yc; da.Prow = Prow; da.Pcol = Pcol;
  da.tile_block = reinterpret_cast<int*>(at(Q.o_tileblk));
  da.tile_first = reinterpret_cast<int*>(at(Q.o_tilefirst));
  da.blk_yoff = reinterpret_cast<int64_t*>(at(Q.o_byoff));
  da.blk_row0 = reinterpret_cast<int*>(at(Q.o_brow0));
  da.blk_col0 = reinterpret_cast<int*>(at(Q.o_bcol0));
  da.blk_nb = reinterpret_cast<int*>(at(Q.o_bnb));
  da.blk_mb = reinterpret_cast<int*>(at(Q.o_bmb));
  da.blk_ldy = reinterpret_cast<int*>(at(Q.o_bldy));
  da.blk_rpw = reinterpret_cast<int*>(at(Q.o_brpw));
  da.blk_nct = reinterpret_cast<int*>(at(Q.o_bnct));
  da.f = family_args(c->cfg);
  da.partial = reinterpret_cast<double*>(at(Q.o_devpartial));
  da.n_tiles = Q.dev_tiles;
  double* scal = reinterpret_cast<double*>(at(Q.o_scal));
  std::vector<double> kproj;
  double kproj_total = 0.0;
  if (dev_trace_host) {
    const int rc = count_constants(P.fam, da, tileblk, P.S, st, kproj, kproj_total);
    if (rc != GMF_OK) return rc;
  }
  auto proj_dev = [&](double* out) -> int {
    HIP_TRY(gmf::launch_deviance(P.fam, P.KP, da, st));
    HIP_TRY(gmf::launch_finalize(da.partial, Q.dev_tiles, nullptr, 0, nullptr, scal, st));
    HIP_TRY(hipMemcpyAsync(out, scal, sizeof(double), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    *out += 2.0 * kproj_total;
    return GMF_OK;
  };
  if (dev_trace_host) {
    const int rc = proj_dev(dev_trace_host);
    if (rc != GMF_OK) return rc;
    if (epoch_ms_host) epoch_ms_host[0] = ms_since(t_start);
  }

  // ---- the row-side steps: one launch per step, each wavefront steps its own
  // rows over the whole column block (project.hip)
  const gmf::LevelArgs la = level_args(c);
  gmf::ProjStepArgs pa{};
  pa.Prow = Prow; pa.Grow = Grow; pa.Hrow = Hrow; pa.n = n_new;
  pa.p = P.p; pa.q = P.q; pa.KU = P.KU;
  pa.lam_A = la.lam_A; pa.lam_U = la.lam_U; pa.a1 = la.a1; pa.a2 = la.a2; pa.damping = la.damping;
  pa.f = la.f; pa.err_flag = la.err_flag;
  for (int e = 0; e < epochs; ++e) {
    for (int k = 0; k < P.S; ++k) {
      const int64_t t = (int64_t)e * P.S + k + 1;
      pa.Y = Yb + (int64_t)n_new * P.coP[k];
      pa.Yc = Yc ? Yc + (int64_t)n_new * P.coP[k] : nullptr;
      pa.ldy = P.ld[k]; pa.m_b = P.mcols[k];
      pa.Pcol = Pcol + (int64_t)P.co[k] * P.KP;
      pa.scale_m = (double)P.m / P.mcols[k];
      pa.stepsize = learning_rate(c->cfg, t) * bias_factor(c->cfg, t);
      HIP_TRY(gmf::launch_project_step(P.prec, P.fam, P.KP, pa, st));
    }
    if (dev_trace_host) {
      const int rc = proj_dev(dev_trace_host + e + 1);
      if (rc != GMF_OK) return rc;
      if (epoch_ms_host) epoch_ms_host[e + 1] = ms_since(t_start);
    }
  }
  const int* iota = reinterpret_cast<int*>(at(Q.o_iota));
  HIP_TRY(gmf::launch_unpack_panel(Prow, P.KP, iota, n_new, P.p, P.q, A_out, st));
  HIP_TRY(gmf::launch_unpack_panel(Prow, P.KP, iota, n_new, P.p + P.q, P.d, U_out, st));
  return check_flag(c);
}

}  // namespace

extern "C" int gmf_project(void* ctx, void* ws, size_t ws_bytes, const void* Ynew, int32_t y_dtype,
                           int64_t n_new, const float* Xnew, const float* A0, const float* U0,
                           int32_t epochs, int32_t frozen, float* A_out, float* U_out,
                           double* dev_trace_host) {
  if (!ctx) return fail(GMF_EINVAL, "ctx is NULL");
  return project_impl(as_ctx(ctx), ws, ws_bytes, Ynew, y_dtype, n_new, Xnew, A0, U0, kInitGiven,
                      nullptr, epochs, frozen, A_out, U_out, dev_trace_host, nullptr, nullptr);
}

extern "C" int gmf_project_warm(void* ctx, void* ws, size_t ws_bytes, const void* Ynew,
                                int32_t y_dtype, int64_t n_new, const float* Xnew,
                                const float* U_cand, int32_t epochs, int32_t frozen, float* A_out,
                                float* U_out, double* dev_trace_host, double* epoch_ms_host,
                                int64_t* fallback_rows_host) {
  if (!ctx) return fail(GMF_EINVAL, "ctx is NULL");
  return project_impl(as_ctx(ctx), ws, ws_bytes, Ynew, y_dtype, n_new, Xnew, nullptr, nullptr,
                      kInitWarm, U_cand, epochs, frozen, A_out, U_out, dev_trace_host,
                      epoch_ms_host, fallback_rows_host);
}

extern "C" int gmf_project_noalloc(void* ctx, const void* Ynew, int32_t y_dtype, int64_t n_new,
                                   const float* Xnew, const float* A0, const float* U0,
                                   int32_t epochs, int32_t frozen, float* A_out, float* U_out,
                                   double* dev_trace_host) {
  if (!ctx) return fail(GMF_EINVAL, "ctx is NULL");
  Ctx* c = as_ctx(ctx);
  void* ws = (c->device >= 0 && c->device < kMaxDevices) ? scratch_addr[c->device] : nullptr;
  if (!ws) return fail(GMF_EDEVICE, "resident scratch of the context's device is not set up");
  ProjPlan Q;
  if (!make_proj_plan(c, n_new, Q)) return fail(GMF_EINVAL, "bad n_new");
  if (Q.total > kScratchBytes)
    return fail(GMF_EWORKSPACE, "projection of " + std::to_string(n_new) + " rows needs " +
                                    std::to_string(Q.total) + " bytes of scratch, more than the " +
                                    std::to_string(kScratchBytes) + " resident bytes");
  return project_impl(c, ws, kScratchBytes, Ynew, y_dtype, n_new, Xnew, A0, U0, kInitGiven,
                      nullptr, epochs, frozen, A_out, U_out, dev_trace_host, nullptr, nullptr);
}

int gmf_set_trace(void* ctx, void* buffer, int64_t records) {
  if (!ctx) return fail(GMF_EINVAL, "ctx is NULL");
  Ctx* c = as_ctx(ctx);
  c->trace = static_cast<unsigned long long*>(buffer);
  c->trace_cap = buffer ? records : 0;
  c->trace_used = 0;
  return GMF_OK;
}

int gmf_set_timing(void* ctx, int32_t enable) {
  if (!ctx) return fail(GMF_EINVAL, "ctx is NULL");
  Ctx* c = as_ctx(ctx);
  if (enable && c->events.empty()) {
    c->timed_kind.assign(kMaxTimedSteps, 0);
    c->events.resize(2 * kMaxTimedSteps);
    for (auto& e : c->events) HIP_TRY(hipEventCreate(&e));
  }
  c->timing = enable != 0;
  return GMF_OK;
}

int gmf_get_timing_by_kind(void* ctx, double* ms_host, double* launches_host) {
  if (!ctx || !ms_host || !launches_host) return fail(GMF_EINVAL, "NULL argument");
  Ctx* c = as_ctx(ctx);
  HIP_TRY(hipStreamSynchronize(c->st));
  ms_host[0] = ms_host[1] = 0.0;
  launches_host[0] = launches_host[1] = 0.0;
  for (int64_t k = 0; k < c->timed_launches; ++k) {
    float ms = 0;
    HIP_TRY(hipEventElapsedTime(&ms, c->events[2 * k], c->events[2 * k + 1]));
    ms_host[c->timed_kind[k]] += ms;
    launches_host[c->timed_kind[k]] += 1.0;
  }
  return GMF_OK;
}

int gmf_get_timing(void* ctx, double* launch_ms_host, double* launches_host,
                   int64_t* steps_host) {
  if (!ctx) return fail(GMF_EINVAL, "ctx is NULL");
  Ctx* c = as_ctx(ctx);
  HIP_TRY(hipStreamSynchronize(c->st));
  double tot = 0;
  for (int64_t k = 0; k < c->timed_launches; ++k) {
    float ms = 0;
    HIP_TRY(hipEventElapsedTime(&ms, c->events[2 * k], c->events[2 * k + 1]));
    tot += ms;
  }
  if (launch_ms_host) *launch_ms_host = tot;
  if (launches_host) *launches_host = (double)c->timed_launches;
  if (steps_host) *steps_host = c->timed_steps;
  c->timed_launches = 0;
  c->timed_steps = 0;
  return GMF_OK;
}

void gmf_destroy(void* ctx) {
  Ctx* c = as_ctx(ctx);
  if (!c) return;
  for (auto& e : c->events) (void)hipEventDestroy(e);
  if (c->side) {
    (void)hipStreamSynchronize(c->side);
    for (auto& e : c->ev_snap) (void)hipEventDestroy(e);
    for (auto& e : c->ev_done) (void)hipEventDestroy(e);
    if (c->ev_start) (void)hipEventDestroy(c->ev_start);
    (void)hipStreamDestroy(c->side);
  }
  delete c;
}

// gmf_run: epochs of steps on the context's stream; every eval_every epochs
// the panels are copied into one of two snapshot buffers and the full
// deviance of the snapshot is formed on a second stream, overlapped with the
// following steps.  A snapshot buffer is reused only after the evaluation
// that read it has finished (the context's stream waits for it).
int gmf_run(void* ctx, int32_t epochs, int32_t eval_every, double* dev_trace_host,
            double* eval_ms_host) {
  if (!ctx) return fail(GMF_EINVAL, "ctx is NULL");
  if (epochs < 0 || eval_every < 1) return fail(GMF_EINVAL, "bad epochs / eval_every");
  if (eval_ms_host && !dev_trace_host) return fail(GMF_EINVAL, "eval_ms_host needs dev_trace_host");
  Ctx* c = as_ctx(ctx);
  const Plan& P = c->P;
  const int64_t per_epoch = (int64_t)P.R * P.S;
  const int nev = dev_trace_host ? epochs / eval_every : 0;
  const bool overlap = c->cfg.eval_overlap != 0;
  hipStream_t es = overlap ? c->side : c->st;   // the evaluations' stream
  if (nev > 0) {
    if (overlap && !c->side) {
      HIP_TRY(hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking));
      es = c->side;
    }
    if (!c->ev_start) HIP_TRY(hipEventCreate(&c->ev_start));
    while ((int)c->ev_done.size() < nev) {
      hipEvent_t a = nullptr, b = nullptr;
      HIP_TRY(hipEventCreateWithFlags(&a, hipEventDisableTiming));
      HIP_TRY(hipEventCreate(&b));
      c->ev_snap.push_back(a);
      c->ev_done.push_back(b);
    }
    HIP_TRY(hipEventRecord(c->ev_start, c->st));
  }
  const size_t snap_elems = (size_t)(P.n + P.m) * P.KP;
  float* snap = c->at<float>(P.o_snap);
  double* part2 = c->at<double>(P.o_devpart2);
  double* evring = c->at<double>(P.o_evring);
  std::vector<double> res(8 * (size_t)std::max(nev, 1));
  int ev_i = 0, drained = 0;
  auto drain = [&](int upto) -> int {   // copy evaluations [drained, upto) to the host
    if (upto <= drained) return GMF_OK;
    HIP_TRY(hipStreamSynchronize(es));
    for (int i = drained; i < upto; ++i)
      HIP_TRY(hipMemcpy(&res[8 * (size_t)i], evring + 8 * (i % kEvRing), 8 * sizeof(double),
                        hipMemcpyDeviceToHost));
    drained = upto;
    return GMF_OK;
  };
  for (int e = 1; e <= epochs; ++e) {
    int rc = enqueue_steps(c, per_epoch);
    if (rc != GMF_OK) return rc;
    if (nev == 0 || e % eval_every != 0 || ev_i >= nev) continue;
    if (ev_i - drained >= kEvRing) {
      rc = drain(ev_i - kEvRing + 1);
      if (rc != GMF_OK) return rc;
    }
    if (!overlap) {   // in order after the epoch's steps, the whole device
      gmf::DevArgs da = dev_args(c);
      da.partial = part2;
      HIP_TRY(gmf::launch_deviance(P.fam, P.KP, da, c->st));
      HIP_TRY(gmf::launch_finalize(da.partial, P.dev_tiles, nullptr, 0, c->at<int>(P.o_flag),
                                   evring + 8 * (ev_i % kEvRing), c->st));
      HIP_TRY(hipEventRecord(c->ev_done[ev_i], c->st));
      ++ev_i;
      continue;
    }
    const int slot = ev_i & 1;
    if (ev_i >= 2) HIP_TRY(hipStreamWaitEvent(c->st, c->ev_done[ev_i - 2], 0));
    float* srow = snap + slot * snap_elems;
    float* scol = srow + (size_t)P.n * P.KP;
    HIP_TRY(hipMemcpyAsync(srow, c->at<float>(P.o_Prow), sizeof(float) * (size_t)P.n * P.KP,
                           hipMemcpyDeviceToDevice, c->st));
    HIP_TRY(hipMemcpyAsync(scol, c->at<float>(P.o_Pcol), sizeof(float) * (size_t)P.m * P.KP,
                           hipMemcpyDeviceToDevice, c->st));
    HIP_TRY(hipEventRecord(c->ev_snap[ev_i], c->st));
    HIP_TRY(hipStreamWaitEvent(c->side, c->ev_snap[ev_i], 0));
    gmf::DevArgs da = dev_args(c);
    da.Prow = srow;
    da.Pcol = scol;
    da.partial = part2 + slot * (size_t)P.dev_tiles;
    da.grid_cap = kDevOverlapWGs;   // leave compute units to the steps running beside it
    HIP_TRY(gmf::launch_deviance(P.fam, P.KP, da, c->side));
    HIP_TRY(gmf::launch_finalize(da.partial, P.dev_tiles, nullptr, 0, c->at<int>(P.o_flag),
                                 evring + 8 * (ev_i % kEvRing), c->side));
    HIP_TRY(hipEventRecord(c->ev_done[ev_i], c->side));
    ++ev_i;
  }
  if (nev > 0) {
    const int rc = drain(ev_i);
    if (rc != GMF_OK) return rc;
    // the context's stream continues after the last evaluation
    HIP_TRY(hipStreamWaitEvent(c->st, c->ev_done[ev_i - 1], 0));
    bool flagged = false;
    for (int i = 0; i < ev_i; ++i) {
      dev_trace_host[i] = res[8 * (size_t)i] + 2.0 * c->ktotal;
      flagged = flagged || res[8 * (size_t)i + 5] != 0.0;
      if (eval_ms_host) {
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, c->ev_start, c->ev_done[i]));
        eval_ms_host[i] = ms;
      }
    }
    if (flagged) return check_flag(c);
  }
  return GMF_OK;
}

}  // extern "C"

// ------------------------------------------------------------ saved state --
// A saved state is a header followed by the device regions that make up the
// iterate of Algorithm 1 between two steps: both panels (the parameters, and
// the covariates, in the context's permuted order), the four float64 moment
// arrays of eq. 12 and the ring of block deviances.  The partitions and the
// row-block draws are functions of (seed, n, m, R, S), recorded in the header
// and checked on load, so the step counter t is the whole schedule cursor.
namespace {
constexpr char kStateMagic[8] = {'G', 'M', 'F', 'S', 'T', 'A', 'T', '1'};
constexpr int kStateRegions = 9;
struct StateHeader {
  char magic[8];
  uint32_t version, nregion;
  int64_t n, m;
  int32_t d, p, q, R, S, family, link, KP;
  uint64_t seed;
  int64_t t, batched_upto;
  double stepsize_params[6];   // rate0, decay, tau, alpha1, alpha2, damping (checked)
  int32_t alpha_col, estimate;  // per-column NB shape set; estimation flags (checked)
  uint64_t region_bytes[kStateRegions];
};

void state_regions(const Ctx* c, size_t off[kStateRegions], size_t bytes[kStateRegions]) {
  const Plan& P = c->P;
  off[0] = P.o_Prow; bytes[0] = sizeof(float) * (size_t)P.n * P.KP;
  off[1] = P.o_Pcol; bytes[1] = sizeof(float) * (size_t)P.m * P.KP;
  off[2] = P.o_Grow; bytes[2] = sizeof(double) * (size_t)P.n * P.KU;
  off[3] = P.o_Hrow; bytes[3] = sizeof(double) * (size_t)P.n * P.KU;
  off[4] = P.o_Gcol; bytes[4] = sizeof(double) * (size_t)P.m * P.KV;
  off[5] = P.o_Hcol; bytes[5] = sizeof(double) * (size_t)P.m * P.KV;
  off[6] = P.o_devring; bytes[6] = sizeof(double) * kDevRing;
  off[7] = P.o_est; bytes[7] = sizeof(double) * 4;   // dispersion / NB shape in use
  off[8] = P.o_alphacol; bytes[8] = sizeof(float) * (size_t)P.m;
}

void fill_header(const Ctx* c, StateHeader& h) {
  std::memset(&h, 0, sizeof(h));
  std::memcpy(h.magic, kStateMagic, 8);
  h.version = 1;
  h.nregion = kStateRegions;
  const gmf_config& f = c->cfg;
  h.n = f.n; h.m = f.m; h.d = f.d; h.p = f.p; h.q = f.q; h.R = f.R; h.S = f.S;
  h.family = f.family; h.link = f.link; h.KP = c->P.KP; h.seed = f.seed;
  h.t = c->t; h.batched_upto = c->batched_upto;
  const double sp[6] = {f.rate0, f.decay, f.tau, f.alpha1, f.alpha2, f.damping};
  std::memcpy(h.stepsize_params, sp, sizeof(sp));
  h.alpha_col = c->alpha_col ? 1 : 0;
  h.estimate = (f.estimate_phi ? 1 : 0) | (f.estimate_alpha ? 2 : 0) | (f.allow_missing ? 4 : 0);
  size_t off[kStateRegions], bytes[kStateRegions];
  state_regions(c, off, bytes);
  for (int i = 0; i < kStateRegions; ++i) h.region_bytes[i] = bytes[i];
}

size_t state_total(const Ctx* c) {
  size_t off[kStateRegions], bytes[kStateRegions];
  state_regions(c, off, bytes);
  size_t tot = sizeof(StateHeader);
  for (int i = 0; i < kStateRegions; ++i) tot += bytes[i];
  return tot;
}
}  // namespace

extern "C" size_t gmf_state_bytes(void* ctx) {
  return ctx ? state_total(as_ctx(ctx)) : 0;
}

extern "C" int gmf_save_state(void* ctx, void* host_buf, size_t bytes) {
  if (!ctx || !host_buf) return fail(GMF_EINVAL, "NULL argument");
  Ctx* c = as_ctx(ctx);
  if (bytes < state_total(c)) return fail(GMF_EINVAL, "buffer smaller than gmf_state_bytes");
  StateHeader h;
  fill_header(c, h);
  char* out = static_cast<char*>(host_buf);
  std::memcpy(out, &h, sizeof(h));
  size_t off[kStateRegions], rb[kStateRegions];
  state_regions(c, off, rb);
  size_t at = sizeof(h);
  for (int i = 0; i < kStateRegions; ++i) {
    HIP_TRY(hipMemcpyAsync(out + at, c->ws + off[i], rb[i], hipMemcpyDeviceToHost, c->st));
    at += rb[i];
  }
  HIP_TRY(hipStreamSynchronize(c->st));
  return check_flag(c);
}

extern "C" int gmf_load_state(void* ctx, const void* host_buf, size_t bytes) {
  if (!ctx || !host_buf) return fail(GMF_EINVAL, "NULL argument");
  Ctx* c = as_ctx(ctx);
  if (bytes < sizeof(StateHeader)) return fail(GMF_EINVAL, "buffer too small for a state header");
  StateHeader h, mine;
  std::memcpy(&h, host_buf, sizeof(h));
  fill_header(c, mine);
  if (std::memcmp(h.magic, kStateMagic, 8) != 0 || h.version != 1 || h.nregion != kStateRegions)
    return fail(GMF_EINVAL, "not a saved libgmf state (magic or version)");
  if (h.n != mine.n || h.m != mine.m || h.d != mine.d || h.p != mine.p || h.q != mine.q ||
      h.R != mine.R || h.S != mine.S || h.family != mine.family || h.link != mine.link ||
      h.KP != mine.KP || h.seed != mine.seed)
    return fail(GMF_EINVAL, "saved state belongs to a context of another shape, family, panel "
                            "stride or schedule seed");
  if (std::memcmp(h.stepsize_params, mine.stepsize_params, sizeof(h.stepsize_params)) != 0)
    return fail(GMF_EINVAL, "saved state was made with other step-size or EMA parameters");
  if (h.estimate != mine.estimate)
    return fail(GMF_EINVAL, "saved state was made with other estimation or missing-entry settings");
  if (h.alpha_col && c->cfg.precision != GMF_PREC_FP32)
    return fail(GMF_EINVAL, "a state with per-column NB shapes needs an FP32 context");
  for (int i = 0; i < kStateRegions; ++i)
    if (h.region_bytes[i] != mine.region_bytes[i]) return fail(GMF_EINVAL, "region size mismatch");
  if (bytes < state_total(c)) return fail(GMF_EINVAL, "buffer shorter than the saved state");
  if (h.t < 0 || h.batched_upto < 0 || h.batched_upto > h.t)
    return fail(GMF_EINVAL, "corrupt step counter");
  size_t off[kStateRegions], rb[kStateRegions];
  state_regions(c, off, rb);
  const char* in = static_cast<const char*>(host_buf);
  size_t at = sizeof(h);
  for (int i = 0; i < kStateRegions; ++i) {
    HIP_TRY(hipMemcpyAsync(c->ws + off[i], in + at, rb[i], hipMemcpyHostToDevice, c->st));
    at += rb[i];
  }
  HIP_TRY(hipStreamSynchronize(c->st));
  c->t = h.t;
  c->batched_upto = h.batched_upto;
  if (h.alpha_col && !c->alpha_col) {
    c->alpha_col = true;
    c->P.fam = gmf::kGeneric;
  }
  if (h.alpha_col || c->cfg.estimate_alpha) {
    const int rc = count_constants(c->P.fam, dev_args(c), dev_tile_blocks(c->P), c->P.R * c->P.S,
                                   c->st, c->kblock, c->ktotal);
    if (rc != GMF_OK) return rc;
  }
  return check_flag(c);
}

extern "C" int gmf_set_column_alpha(void* ctx, const float* alpha) {
  if (!ctx || !alpha) return fail(GMF_EINVAL, "NULL argument");
  Ctx* c = as_ctx(ctx);
  Plan& P = c->P;
  if (c->cfg.family != GMF_NEGBIN) return fail(GMF_EINVAL, "per-column shapes need the NB family");
  if (c->cfg.estimate_alpha) return fail(GMF_EINVAL, "the NB shape is being estimated");
  if (P.prec != GMF_PREC_FP32)
    return fail(GMF_EINVAL, "per-column NB shapes run in FP32 precision (gmf_set_precision)");
  // caller order -> permuted order, validated on the device
  HIP_TRY(gmf::launch_pack_panel(alpha, 1, nullptr, 0, nullptr, 0, c->at<int>(P.o_colperm), P.m, 1,
                                 c->at<float>(P.o_alphacol), c->st));
  HIP_TRY(gmf::launch_check_positive(c->at<float>(P.o_alphacol), P.m, c->at<int>(P.o_flag), c->st));
  const int rc0 = check_flag(c);
  if (rc0 != GMF_OK) return rc0;
  c->alpha_col = true;
  P.fam = gmf::kGeneric;
  return count_constants(P.fam, dev_args(c), dev_tile_blocks(P), P.R * P.S, c->st, c->kblock,
                         c->ktotal);
}

extern "C" int gmf_get_dispersion(void* ctx, double* phi_host, double* alpha_host) {
  if (!ctx) return fail(GMF_EINVAL, "ctx is NULL");
  double d[2];
  const int rc = current_dispersion(as_ctx(ctx), d);
  if (rc != GMF_OK) return rc;
  if (phi_host) *phi_host = d[0];
  if (alpha_host) *alpha_host = d[1];
  return check_flag(as_ctx(ctx));
}

extern "C" int gmf_heldout_metrics(void* ctx, const void* Ytest, int32_t y_dtype,
                                   double* out_host) {
  if (!ctx || !Ytest || !out_host) return fail(GMF_EINVAL, "NULL argument");
  if (y_dtype != GMF_Y_INT32 && y_dtype != GMF_Y_FLOAT32) return fail(GMF_EINVAL, "bad y_dtype");
  Ctx* c = as_ctx(ctx);
  const Plan& P = c->P;
  double* part = c->at<double>(P.o_hopart);
  // the mean of the observed training entries
  gmf::DevArgs da = dev_args(c);
  HIP_TRY(gmf::launch_observed_sum(da, part, c->st));
  std::vector<double> h(2 * (size_t)P.dev_tiles);
  HIP_TRY(hipMemcpyAsync(h.data(), part, sizeof(double) * h.size(), hipMemcpyDeviceToHost, c->st));
  HIP_TRY(hipStreamSynchronize(c->st));
  double sy = 0.0, cnt = 0.0;
  for (int t = 0; t < P.dev_tiles; ++t) {
    sy += h[2 * t];
    cnt += h[2 * t + 1];
  }
  if (!(cnt > 0)) return fail(GMF_EINVAL, "no observed training entries");
  const double ybar = sy / cnt;
  gmf::HeldoutArgs a{};
  a.Ytest = Ytest;
  a.y_int = y_dtype == GMF_Y_INT32;
  a.Prow = c->at<float>(P.o_Prow);
  a.Pcol = c->at<float>(P.o_Pcol);
  a.KP = P.KP;
  a.row_perm = c->at<int>(P.o_rowperm);
  a.col_perm = c->at<int>(P.o_colperm);
  a.n = P.n;
  a.m = P.m;
  a.ybar = ybar;
  a.f = family_args(c);
  a.partial = part;
  HIP_TRY(gmf::launch_heldout(a, c->st));
  std::vector<double> g(8 * (size_t)P.ho_wg);
  HIP_TRY(hipMemcpyAsync(g.data(), part, sizeof(double) * g.size(), hipMemcpyDeviceToHost, c->st));
  HIP_TRY(hipStreamSynchronize(c->st));
  double s[7] = {0, 0, 0, 0, 0, 0, 0};
  for (int w = 0; w < P.ho_wg; ++w)
    for (int q = 0; q < 7; ++q) s[q] += g[8 * (size_t)w + q];
  out_host[0] = s[1] > 0 ? s[0] / s[1] : 0.0;   // relative squared log error
  out_host[1] = s[3] > 0 ? s[2] / s[3] : 0.0;   // relative Poisson deviance
  out_host[2] = s[5] > 0 ? s[4] / s[5] : 0.0;   // relative deviance of the family
  out_host[3] = s[6];                           // held-out entries
  out_host[4] = ybar;                           // mean of the training entries
  out_host[5] = cnt;                            // observed training entries
  return check_flag(c);
}


// --------------------------------------------------------- initialization --
// The paper's initialization (Section 4.1, least-squares form): OLS column
// effects on L = g(y + c), OLS row effects on the residual given those
// offsets, the leading left singular vectors of the Pearson (or deviance)
// residual matrix at mu~ = g^-1(X B' + Gamma Z') by a randomized range finder
// with power iterations from the caller's test matrix, OLS loadings of the
// link-scale residual on those scores, and equal norms within each pair
// (u_k, v_k).  Every n x m quantity is formed entry by entry inside the passes
// of init.hip; the k x k algebra (Cholesky factors, the symmetric eigenproblem
// of the range finder's small matrix) runs in float64 on the host.
namespace {

constexpr int kInitChunkRows = 1024;
constexpr int kGramParts = 128;

struct InitPlan {
  int kmax = 0, nrt = 0, nct = 0, nch = 0;
  std::vector<int> rt, ct, ch;   // row tiles (r, li0), column tiles (s, lj0), chunks (r, li0, rows)
  size_t o_rt, o_ct, o_ch, o_part, o_Dn, o_Dn2, o_Fn, o_Dm, o_Dm2, o_Fm, o_gpart, o_G, o_M, o_scale,
      o_colfill, total;
};

bool make_init_plan(const Ctx* c, int k, InitPlan& I) {
  const Plan& P = c->P;
  if (k < P.d || k > 64) return false;
  I.kmax = std::max(k, std::max(P.p, P.q));
  I.rt.clear(); I.ct.clear(); I.ch.clear();
  for (int r = 0; r < P.R; ++r)
    for (int li = 0; li < P.nrows[r]; li += 64) { I.rt.push_back(r); I.rt.push_back(li); }
  for (int s = 0; s < P.S; ++s)
    for (int lj = 0; lj < P.mcols[s]; lj += 64) { I.ct.push_back(s); I.ct.push_back(lj); }
  for (int r = 0; r < P.R; ++r)
    for (int li = 0; li < P.nrows[r]; li += kInitChunkRows) {
      I.ch.push_back(r); I.ch.push_back(li); I.ch.push_back(std::min(kInitChunkRows, P.nrows[r] - li));
    }
  I.nrt = (int)I.rt.size() / 2; I.nct = (int)I.ct.size() / 2; I.nch = (int)I.ch.size() / 3;
  const int64_t part_floats = std::max<int64_t>((int64_t)P.S * P.n, (int64_t)I.nch * P.m) * I.kmax;
  size_t o = 0;
  auto take = [&](size_t bytes) { size_t at = o; o = align256(o + bytes); return at; };
  I.o_rt = take(sizeof(int) * I.rt.size());
  I.o_ct = take(sizeof(int) * I.ct.size());
  I.o_ch = take(sizeof(int) * I.ch.size());
  I.o_part = take(sizeof(float) * (size_t)part_floats);
  I.o_Dn = take(sizeof(double) * (size_t)P.n * I.kmax);
  I.o_Dn2 = take(sizeof(double) * (size_t)P.n * I.kmax);
  I.o_Fn = take(sizeof(float) * (size_t)P.n * I.kmax);
  I.o_Dm = take(sizeof(double) * (size_t)P.m * I.kmax);
  I.o_Dm2 = take(sizeof(double) * (size_t)P.m * I.kmax);
  I.o_Fm = take(sizeof(float) * (size_t)P.m * I.kmax);
  I.o_gpart = take(sizeof(double) * kGramParts * 64 * 64);
  I.o_G = take(sizeof(double) * 64 * 64);
  I.o_M = take(sizeof(double) * 64 * 64);
  I.o_scale = take(sizeof(double) * 64);
  I.o_colfill = take(sizeof(float) * (size_t)P.m);
  I.total = o;
  return true;
}

// G = R'R with R upper triangular (k x k, row-major); false if G is not
// positive definite.
bool cholesky_upper(const std::vector<double>& G, int k, std::vector<double>& R) {
  R.assign((size_t)k * k, 0.0);
  for (int j = 0; j < k; ++j) {
    double s = G[(size_t)j * k + j];
    for (int i = 0; i < j; ++i) s -= R[(size_t)i * k + j] * R[(size_t)i * k + j];
    if (!(s > 0.0)) return false;
    const double rjj = std::sqrt(s);
    R[(size_t)j * k + j] = rjj;
    for (int l = j + 1; l < k; ++l) {
      double t = G[(size_t)j * k + l];
      for (int i = 0; i < j; ++i) t -= R[(size_t)i * k + j] * R[(size_t)i * k + l];
      R[(size_t)j * k + l] = t / rjj;
    }
  }
  return true;
}

// Inverse of an upper triangular matrix (back substitution, column by column).
void upper_inverse(const std::vector<double>& R, int k, std::vector<double>& Ri) {
  Ri.assign((size_t)k * k, 0.0);
  for (int j = 0; j < k; ++j) {
    Ri[(size_t)j * k + j] = 1.0 / R[(size_t)j * k + j];
    for (int i = j - 1; i >= 0; --i) {
      double s = 0.0;
      for (int l = i + 1; l <= j; ++l) s += R[(size_t)i * k + l] * Ri[(size_t)l * k + j];
      Ri[(size_t)i * k + j] = -s / R[(size_t)i * k + i];
    }
  }
}

// Eigenvalues (descending) and eigenvectors (columns of V, row-major k x k) of
// a symmetric matrix by cyclic Jacobi rotations.
void sym_eigen(std::vector<double> A, int k, std::vector<double>& ev, std::vector<double>& V) {
  V.assign((size_t)k * k, 0.0);
  for (int i = 0; i < k; ++i) V[(size_t)i * k + i] = 1.0;
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int i = 0; i < k; ++i)
      for (int j = 0; j < k; ++j) {
        const double a = A[(size_t)i * k + j] * A[(size_t)i * k + j];
        tot += a;
        if (i != j) off += a;
      }
    if (off <= 1e-30 * tot) break;
    for (int p = 0; p < k - 1; ++p)
      for (int q = p + 1; q < k; ++q) {
        const double apq = A[(size_t)p * k + q];
        if (apq == 0.0) continue;
        const double app = A[(size_t)p * k + p], aqq = A[(size_t)q * k + q];
        const double theta = (aqq - app) / (2.0 * apq);
        const double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
        const double cs = 1.0 / std::sqrt(t * t + 1.0), sn = t * cs;
        for (int l = 0; l < k; ++l) {   // A <- A J (columns p, q)
          const double alp = A[(size_t)l * k + p], alq = A[(size_t)l * k + q];
          A[(size_t)l * k + p] = cs * alp - sn * alq;
          A[(size_t)l * k + q] = sn * alp + cs * alq;
        }
        for (int l = 0; l < k; ++l) {   // A <- J' A (rows p, q)
          const double apl = A[(size_t)p * k + l], aql = A[(size_t)q * k + l];
          A[(size_t)p * k + l] = cs * apl - sn * aql;
          A[(size_t)q * k + l] = sn * apl + cs * aql;
        }
        for (int l = 0; l < k; ++l) {   // V <- V J
          const double vlp = V[(size_t)l * k + p], vlq = V[(size_t)l * k + q];
          V[(size_t)l * k + p] = cs * vlp - sn * vlq;
          V[(size_t)l * k + q] = sn * vlp + cs * vlq;
        }
      }
  }
  std::vector<int> order(k);
  for (int i = 0; i < k; ++i) order[i] = i;
  std::sort(order.begin(), order.end(),
            [&](int a, int b) { return A[(size_t)a * k + a] > A[(size_t)b * k + b]; });
  ev.resize(k);
  std::vector<double> Vs((size_t)k * k);
  for (int j = 0; j < k; ++j) {
    ev[j] = A[(size_t)order[j] * k + order[j]];
    for (int i = 0; i < k; ++i) Vs[(size_t)i * k + j] = V[(size_t)i * k + order[j]];
  }
  V.swap(Vs);
}

struct InitRun {
  Ctx* c;
  InitPlan I;
  char* W;
  template <class T> T* at(size_t off) const { return reinterpret_cast<T*>(W + off); }

  gmf::InitPassArgs pass_args(int mode, int ke, float c_off, const float* Q, int kq,
                              int64_t nout) const {
    const Plan& P = c->P;
    gmf::InitPassArgs a{};
    a.Yb = c->at<float>(P.o_Yb);
    a.Wb = P.with_w ? c->at<float>(P.o_Wb) : nullptr;
    a.LDtot = P.LDtot;
    a.Prow = c->at<float>(P.o_Prow);
    a.Pcol = c->at<float>(P.o_Pcol);
    a.KP = P.KP; a.ke = ke;
    a.ro = c->at<int>(P.o_ro); a.nrows = c->at<int>(P.o_nrows);
    a.co = c->at<int>(P.o_co); a.mcols = c->at<int>(P.o_mcols);
    a.ldy = c->at<int>(P.o_ld); a.coP = c->at<int64_t>(P.o_coP);
    a.mode = mode; a.fam = P.fam; a.log_link = c->cfg.link == GMF_LINK_LOG;
    a.c_off = c_off;
    a.f = family_args(c);
    a.colfill = nullptr;
    a.Q = Q; a.kq = kq;
    a.part = at<float>(I.o_part);
    a.nout = nout;
    return a;
  }
  // E Q over all column blocks: out (n x kq) = sum over s of the partials.
  int row_pass(int mode, int ke, float c_off, const float* Qm, int kq, double* out64, float* out32) {
    const Plan& P = c->P;
    gmf::InitPassArgs a = pass_args(mode, ke, c_off, Qm, kq, P.n);
    a.tiles = at<int>(I.o_rt);
    HIP_TRY(gmf::launch_init_pass(a, true, I.nrt, P.S, c->st));
    HIP_TRY(gmf::launch_sum_parts(a.part, P.S, P.n * kq, P.n * kq, out64, out32, c->st));
    return GMF_OK;
  }
  // E' Q over all row chunks: out (m x kq).
  int col_pass(int mode, int ke, float c_off, const float* Qn, int kq, double* out64, float* out32,
               const float* colfill = nullptr) {
    const Plan& P = c->P;
    gmf::InitPassArgs a = pass_args(mode, ke, c_off, Qn, kq, P.m);
    a.tiles = at<int>(I.o_ct);
    a.chunks = at<int>(I.o_ch);
    a.colfill = colfill;
    HIP_TRY(gmf::launch_init_pass(a, false, I.nct, I.nch, c->st));
    HIP_TRY(gmf::launch_sum_parts(a.part, I.nch, P.m * kq, P.m * kq, out64, out32, c->st));
    return GMF_OK;
  }
  // k x k Gram matrix A'A of a tall float64 operand, on the host.
  int gram(const double* A, int64_t rows, int k, std::vector<double>& G) {
    HIP_TRY(gmf::launch_gram(A, rows, k, at<double>(I.o_gpart), kGramParts, at<double>(I.o_G), c->st));
    G.resize((size_t)k * k);
    HIP_TRY(hipMemcpyAsync(G.data(), at<double>(I.o_G), sizeof(double) * G.size(),
                           hipMemcpyDeviceToHost, c->st));
    HIP_TRY(hipStreamSynchronize(c->st));
    return GMF_OK;
  }
  // Copies a small host matrix to the device and waits, so that the host
  // buffer may be released at once.
  int upload_small(const std::vector<double>& M, size_t off) {
    HIP_TRY(hipMemcpyAsync(at<double>(off), M.data(), sizeof(double) * M.size(),
                           hipMemcpyHostToDevice, c->st));
    HIP_TRY(hipStreamSynchronize(c->st));
    return GMF_OK;
  }
  // A (rows x k, float64, in place through Tmp) <- an orthonormal basis of its
  // range, by two rounds of Cholesky QR; the float32 copy goes to out32.
  int orth(double* A, double* Tmp, int64_t rows, int k, float* out32) {
    for (int round = 0; round < 2; ++round) {
      std::vector<double> G, R, Ri;
      int rc = gram(A, rows, k, G);
      if (rc != GMF_OK) return rc;
      if (!cholesky_upper(G, k, R))
        return fail(GMF_ENUMERIC, "initialization: the range finder's basis lost rank");
      upper_inverse(R, k, Ri);
      rc = upload_small(Ri, I.o_M);
      if (rc != GMF_OK) return rc;
      HIP_TRY(gmf::launch_apply(A, rows, k, k, at<double>(I.o_M), nullptr, Tmp,
                                round == 1 ? out32 : nullptr, nullptr, 0, 0, c->st));
      HIP_TRY(hipMemcpyAsync(A, Tmp, sizeof(double) * rows * k, hipMemcpyDeviceToDevice, c->st));
    }
    return GMF_OK;
  }
  // (A'A)^-1 for a tall operand A (rows x k).
  int normal_inverse(const double* A, int64_t rows, int k, std::vector<double>& Inv) {
    std::vector<double> G, R, Ri;
    int rc = gram(A, rows, k, G);
    if (rc != GMF_OK) return rc;
    if (!cholesky_upper(G, k, R))
      return fail(GMF_ENUMERIC, "initialization: a design Gram matrix is not positive definite");
    upper_inverse(R, k, Ri);
    Inv.assign((size_t)k * k, 0.0);
    for (int i = 0; i < k; ++i)
      for (int j = 0; j < k; ++j) {
        double s = 0.0;
        for (int l = std::max(i, j); l < k; ++l) s += Ri[(size_t)i * k + l] * Ri[(size_t)j * k + l];
        Inv[(size_t)i * k + j] = s;
      }
    return GMF_OK;
  }
};

}  // namespace

extern "C" size_t gmf_initialize_workspace_bytes(void* ctx, int32_t k) {
  if (!ctx) return 0;
  InitPlan I;
  if (!make_init_plan(as_ctx(ctx), k, I)) return 0;
  return I.total;
}

extern "C" int gmf_initialize(void* ctx, void* ws, size_t ws_bytes, const float* Omega, int32_t k,
                              int32_t power_iters, int32_t residual, double y_offset) {
  if (!ctx) return fail(GMF_EINVAL, "ctx is NULL");
  Ctx* c = as_ctx(ctx);
  const Plan& P = c->P;
  InitRun run;
  run.c = c;
  if (!make_init_plan(c, k, run.I)) return fail(GMF_EINVAL, "k must be in [d, 64]");
  const InitPlan& I = run.I;
  if (!Omega) return fail(GMF_EINVAL, "Omega is NULL");
  if (power_iters < 0 || power_iters > 64) return fail(GMF_EINVAL, "power_iters must be in [0, 64]");
  if (residual != 0 && residual != 1) return fail(GMF_EINVAL, "residual must be 0 (Pearson) or 1 (deviance)");
  if (P.p + P.q > 32) return fail(GMF_EINVAL, "initialization needs p + q <= 32");
  if (c->t != 0) return fail(GMF_EINVAL, "initialization must precede the first step");
  if (!ws || (reinterpret_cast<uintptr_t>(ws) & 255) != 0 || ws_bytes < I.total)
    return fail(GMF_EWORKSPACE, "initialization workspace NULL, misaligned or smaller than " +
                                    std::to_string(I.total) + " bytes");
  run.W = static_cast<char*>(ws);
  const float c_off = (float)(y_offset >= 0 ? y_offset : (c->cfg.link == GMF_LINK_IDENTITY ? 0.0 : 0.5));
  if (c->cfg.link != GMF_LINK_IDENTITY && !(c_off > 0))
    return fail(GMF_EINVAL, "the log and logit links need y_offset > 0");
  hipStream_t st = c->st;
  float* Prow = c->at<float>(P.o_Prow);
  float* Pcol = c->at<float>(P.o_Pcol);
  HIP_TRY(hipMemcpyAsync(run.at<int>(I.o_rt), I.rt.data(), sizeof(int) * I.rt.size(), hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(run.at<int>(I.o_ct), I.ct.data(), sizeof(int) * I.ct.size(), hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(run.at<int>(I.o_ch), I.ch.data(), sizeof(int) * I.ch.size(), hipMemcpyHostToDevice, st));
  // start from B = Gamma = U = V = 0 (X and Z stay)
  if (P.p > 0) HIP_TRY(gmf::launch_panel_cols(Pcol, P.KP, P.m, 0, P.p, nullptr, nullptr, 1, st));
  if (P.q > 0) HIP_TRY(gmf::launch_panel_cols(Prow, P.KP, P.n, P.p, P.q, nullptr, nullptr, 1, st));
  HIP_TRY(gmf::launch_panel_cols(Prow, P.KP, P.n, P.p + P.q, P.d, nullptr, nullptr, 1, st));
  HIP_TRY(gmf::launch_panel_cols(Pcol, P.KP, P.m, P.p + P.q, P.d, nullptr, nullptr, 1, st));
  double* Dn = run.at<double>(I.o_Dn);
  double* Dn2 = run.at<double>(I.o_Dn2);
  float* Fn = run.at<float>(I.o_Fn);
  double* Dm = run.at<double>(I.o_Dm);
  double* Dm2 = run.at<double>(I.o_Dm2);
  float* Fm = run.at<float>(I.o_Fm);
  int rc = GMF_OK;
  std::vector<double> Inv;
  // missing entries of L take their column's mean of the observed L (the
  // prediction before any effect is fitted)
  const float* colfill = nullptr;
  if (c->cfg.allow_missing) {
    HIP_TRY(gmf::launch_fill_i32(reinterpret_cast<int*>(Fn), P.n, 0x3f800000, st));   // ones
    rc = run.col_pass(0, 0, c_off, Fn, 1, Dm, nullptr);       // sums of the observed L
    if (rc != GMF_OK) return rc;
    rc = run.col_pass(4, 0, c_off, Fn, 1, Dm2, nullptr);      // observed counts
    if (rc != GMF_OK) return rc;
    HIP_TRY(gmf::launch_ratio(Dm, Dm2, P.m, run.at<float>(I.o_colfill), st));
    colfill = run.at<float>(I.o_colfill);
  }
  // 1. column effects: B' = (X'X)^-1 X'L
  if (P.p > 0) {
    HIP_TRY(gmf::launch_panel_cols(Prow, P.KP, P.n, 0, P.p, Dn, Fn, 0, st));
    rc = run.col_pass(0, 0, c_off, Fn, P.p, Dm, nullptr, colfill);
    if (rc != GMF_OK) return rc;
    rc = run.normal_inverse(Dn, P.n, P.p, Inv);
    if (rc != GMF_OK) return rc;
    rc = run.upload_small(Inv, I.o_M);
    if (rc != GMF_OK) return rc;
    HIP_TRY(gmf::launch_apply(Dm, P.m, P.p, P.p, run.at<double>(I.o_M), nullptr, nullptr, nullptr,
                              Pcol, P.KP, 0, st));
  }
  // 2. row effects given the column offsets: Gamma = (L - X B') Z (Z'Z)^-1
  if (P.q > 0) {
    HIP_TRY(gmf::launch_panel_cols(Pcol, P.KP, P.m, P.p, P.q, Dm, Fm, 0, st));
    rc = run.row_pass(1, P.p, c_off, Fm, P.q, Dn, nullptr);
    if (rc != GMF_OK) return rc;
    rc = run.normal_inverse(Dm, P.m, P.q, Inv);
    if (rc != GMF_OK) return rc;
    rc = run.upload_small(Inv, I.o_M);
    if (rc != GMF_OK) return rc;
    HIP_TRY(gmf::launch_apply(Dn, P.n, P.q, P.q, run.at<double>(I.o_M), nullptr, nullptr, nullptr,
                              Prow, P.KP, P.p, st));
  }
  // 3. scores: randomized range finder on the residual matrix E
  const int ke = P.p + P.q;
  const int emode = residual == 0 ? 2 : 3;
  HIP_TRY(gmf::launch_pack_panel(Omega, k, nullptr, 0, nullptr, 0, c->at<int>(P.o_colperm), P.m, k,
                                 Fm, st));
  rc = run.row_pass(emode, ke, c_off, Fm, k, Dn, nullptr);          // Y = E Omega
  if (rc != GMF_OK) return rc;
  for (int it = 0; it < power_iters; ++it) {
    rc = run.orth(Dn, Dn2, P.n, k, Fn);
    if (rc != GMF_OK) return rc;
    rc = run.col_pass(emode, ke, c_off, Fn, k, Dm, nullptr);        // E' Q
    if (rc != GMF_OK) return rc;
    rc = run.orth(Dm, Dm2, P.m, k, Fm);
    if (rc != GMF_OK) return rc;
    rc = run.row_pass(emode, ke, c_off, Fm, k, Dn, nullptr);        // Y = E orth(E' Q)
    if (rc != GMF_OK) return rc;
  }
  rc = run.orth(Dn, Dn2, P.n, k, Fn);                                 // Q
  if (rc != GMF_OK) return rc;
  rc = run.col_pass(emode, ke, c_off, Fn, k, Dm, nullptr);          // (Q'E)' = E'Q
  if (rc != GMF_OK) return rc;
  {
    // left singular vectors of Q'E = eigenvectors of (Q'E)(Q'E)' = (E'Q)'(E'Q)
    std::vector<double> G2, ev, Vk;
    rc = run.gram(Dm, P.m, k, G2);
    if (rc != GMF_OK) return rc;
    sym_eigen(G2, k, ev, Vk);
    c->init_sv.resize(k);
    for (int j = 0; j < k; ++j) c->init_sv[j] = std::sqrt(std::max(ev[j], 0.0));
    std::vector<double> Ub((size_t)k * P.d);
    for (int i = 0; i < k; ++i)
      for (int j = 0; j < P.d; ++j) Ub[(size_t)i * P.d + j] = Vk[(size_t)i * k + j];
    rc = run.upload_small(Ub, I.o_M);
    if (rc != GMF_OK) return rc;
    HIP_TRY(gmf::launch_apply(Dn, P.n, k, P.d, run.at<double>(I.o_M), nullptr, Dn2, Fn, nullptr, 0,
                              0, st));                              // U = Q Ub
  }
  // 4. loadings: V = R' U (U'U)^-1 with R = L - X B' - Gamma Z'
  rc = run.col_pass(1, ke, c_off, Fn, P.d, Dm, nullptr);
  if (rc != GMF_OK) return rc;
  std::vector<double> GU;
  rc = run.gram(Dn2, P.n, P.d, GU);
  if (rc != GMF_OK) return rc;
  rc = run.normal_inverse(Dn2, P.n, P.d, Inv);
  if (rc != GMF_OK) return rc;
  rc = run.upload_small(Inv, I.o_M);
  if (rc != GMF_OK) return rc;
  HIP_TRY(gmf::launch_apply(Dm, P.m, P.d, P.d, run.at<double>(I.o_M), nullptr, Dm2, nullptr, nullptr,
                            0, 0, st));
  // equal norms within each pair: u_k * s_k, v_k / s_k, s_k = sqrt(|v_k| / |u_k|)
  std::vector<double> GV;
  rc = run.gram(Dm2, P.m, P.d, GV);
  if (rc != GMF_OK) return rc;
  std::vector<double> su(P.d), sv(P.d), eye((size_t)P.d * P.d, 0.0);
  for (int j = 0; j < P.d; ++j) {
    eye[(size_t)j * P.d + j] = 1.0;
    const double nu = std::sqrt(GU[(size_t)j * P.d + j]), nv = std::sqrt(GV[(size_t)j * P.d + j]);
    const double s = (nu > 0 && nv > 0) ? std::sqrt(nv / nu) : 1.0;
    su[j] = s;
    sv[j] = 1.0 / s;
  }
  rc = run.upload_small(eye, I.o_M);
  if (rc != GMF_OK) return rc;
  std::vector<double> scales(su);
  scales.insert(scales.end(), sv.begin(), sv.end());
  HIP_TRY(hipMemcpyAsync(run.at<double>(I.o_scale), scales.data(), sizeof(double) * scales.size(),
                         hipMemcpyHostToDevice, st));
  HIP_TRY(hipStreamSynchronize(st));
  HIP_TRY(gmf::launch_apply(Dn2, P.n, P.d, P.d, run.at<double>(I.o_M), run.at<double>(I.o_scale),
                            nullptr, nullptr, Prow, P.KP, P.p + P.q, st));
  HIP_TRY(gmf::launch_apply(Dm2, P.m, P.d, P.d, run.at<double>(I.o_M), run.at<double>(I.o_scale) + P.d,
                            nullptr, nullptr, Pcol, P.KP, P.p + P.q, st));
  HIP_TRY(hipStreamSynchronize(st));
  return check_flag(c);
}


// ------------------------------------------------------------ batched fits --
// Many independent fits advanced together.  One epoch of the batch is a fixed
// sequence of launches: for k = 0 .. L-1, the tiles of step k of every fit
// that has one (one segment per fit), then the updates of step k, then one
// workgroup that advances the epoch cursor.  Each fit's steps follow one
// another exactly as in gmf_step (its tiles of step k run after the updates
// of step k-1, in the previous launch); the fits run side by side.  The
// launch sequence does not depend on the random row blocks: those (and the
// step sizes) come from a device table of `table_epochs` epochs refilled from
// the host, so one recorded sequence (a HIP graph when asked for) serves every
// epoch.
namespace {

struct BatchLaunch {
  int seg0, nsegs, grid;
  bool updates_only;   // no tile segment: the update-only kernel
};

struct Batch {
  std::vector<Ctx*> fits;
  int prec = 0, KP = 0;
  hipStream_t st = nullptr;
  hipEvent_t ev = nullptr;
  int table_epochs = 1;
  int64_t steps_per_epoch = 0;
  std::vector<int64_t> step_off;     // per fit: offset of its steps inside an epoch
  int L = 0;                         // most steps per epoch over the fits
  gmf::LevelArgs* fits_dev = nullptr;
  gmf::BatchSeg* segs_dev = nullptr;
  gmf::LevelStep* steps_dev = nullptr;
  int* cursor = nullptr;
  double* scal = nullptr;            // 8 doubles per fit
  std::vector<BatchLaunch> launches;
  bool use_graph = false;
  int mode = 0;                      // 0 fixed sequence, 1 its graph, 2 level placement
  std::vector<int> tile_wgs, upd_wgs;   // per fit: workgroups of a step's tiles / updates
  std::vector<gmf::BatchSeg> host_segs; // level placement: the segments of the current table
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int64_t used = 0, valid = 0;       // epochs of the current table consumed / available
  std::vector<gmf::LevelStep> host_steps;
};

struct BatchSizes {
  int L = 0;
  int64_t steps_per_epoch = 0;
  size_t o_fits = 0, o_segs = 0, o_steps = 0, o_cursor = 0, o_scal = 0, total = 0;
};

bool batch_sizes(void* const* ctxs, int nfits, int table_epochs, BatchSizes& z) {
  if (!ctxs || nfits < 1 || table_epochs < 1) return false;
  for (int f = 0; f < nfits; ++f) {
    if (!ctxs[f]) return false;
    const Plan& P = as_ctx(ctxs[f])->P;
    z.L = std::max(z.L, P.R * P.S);
    z.steps_per_epoch += (int64_t)P.R * P.S;
  }
  size_t o = 0;
  auto take = [&](size_t bytes) { size_t at = o; o = align256(o + bytes); return at; };
  z.o_fits = take(sizeof(gmf::LevelArgs) * (size_t)nfits);
  // the fixed sequence: 2 segments per step index and fit; level placement:
  // 2 per step of the table
  z.o_segs = take(sizeof(gmf::BatchSeg) *
                  std::max<size_t>(2 * (size_t)z.L * nfits,
                                   2 * (size_t)z.steps_per_epoch * table_epochs));
  z.o_steps = take(sizeof(gmf::LevelStep) * (size_t)table_epochs * z.steps_per_epoch);
  z.o_cursor = take(sizeof(int) * 4);
  z.o_scal = take(sizeof(double) * 8 * (size_t)nfits);
  z.total = o;
  return true;
}

int enqueue_batch_epoch(Batch* b) {
  for (const BatchLaunch& l : b->launches) {
    gmf::BatchArgs ba;
    ba.fits = b->fits_dev;
    ba.segs = b->segs_dev + l.seg0;
    ba.nsegs = l.nsegs;
    ba.steps = b->steps_dev;
    ba.steps_per_epoch = b->steps_per_epoch;
    ba.table_epochs = b->table_epochs;
    ba.cursor = b->cursor;
    HIP_TRY(gmf::launch_batch(b->prec, b->KP, ba, l.grid, b->st, l.updates_only));
  }
  HIP_TRY(gmf::launch_advance_cursor(b->cursor, b->st));
  return GMF_OK;
}

// Level placement of the table's `ne` epochs (mode 2): each fit's steps get
// the level rule of a single fit, T(t) = 2 + the largest level of the previous
// step on its row block, its column block and its partial slot; launch k runs
// the tiles of every fit's level-k steps and the updates of every fit's
// level-(k-1) steps.  Each fit's steps keep their order and dependencies, so
// the results equal stepping the fits one by one.
int enqueue_batch_leveled(Batch* b, int ne) {
  const int nf = (int)b->fits.size();
  std::vector<std::vector<std::vector<int>>> by_level(nf);
  int max_level = 0;
  for (int f = 0; f < nf; ++f) {
    const Plan& P = b->fits[f]->P;
    const int rs = P.R * P.S;
    std::vector<int> lr(P.R, -1), ls(P.S, -1), lslot(P.nslot, -1);
    for (int k = 0; k < ne * rs; ++k) {
      const int idx = (int)((int64_t)(k / rs) * b->steps_per_epoch + b->step_off[f] + (k % rs));
      const gmf::LevelStep& st = b->host_steps[idx];
      int lv = 0;
      if (lr[st.r] >= 0) lv = std::max(lv, lr[st.r] + 2);
      if (ls[st.s] >= 0) lv = std::max(lv, ls[st.s] + 2);
      if (lslot[st.slot] >= 0) lv = std::max(lv, lslot[st.slot] + 2);
      lr[st.r] = ls[st.s] = lslot[st.slot] = lv;
      if ((int)by_level[f].size() <= lv) by_level[f].resize(lv + 1);
      by_level[f][lv].push_back(idx);
      max_level = std::max(max_level, lv);
    }
  }
  b->host_segs.clear();
  std::vector<BatchLaunch> launches;
  for (int lv = 0; lv <= max_level + 1; ++lv) {
    BatchLaunch l{(int)b->host_segs.size(), 0, 0, true};
    for (int f = 0; f < nf; ++f)
      if (lv < (int)by_level[f].size())
        for (int idx : by_level[f][lv]) {
          b->host_segs.push_back(gmf::BatchSeg{l.grid, f, 0, idx});
          l.grid += b->tile_wgs[f];
          ++l.nsegs;
          l.updates_only = false;
        }
    for (int f = 0; f < nf; ++f)
      if (lv >= 1 && lv - 1 < (int)by_level[f].size())
        for (int idx : by_level[f][lv - 1]) {
          b->host_segs.push_back(gmf::BatchSeg{l.grid, f, 1, idx});
          l.grid += b->upd_wgs[f];
          ++l.nsegs;
        }
    if (l.nsegs > 0) launches.push_back(l);
  }
  HIP_TRY(hipMemcpyAsync(b->segs_dev, b->host_segs.data(), sizeof(gmf::BatchSeg) * b->host_segs.size(),
                         hipMemcpyHostToDevice, b->st));
  for (const BatchLaunch& l : launches) {
    gmf::BatchArgs ba;
    ba.fits = b->fits_dev;
    ba.segs = b->segs_dev + l.seg0;
    ba.nsegs = l.nsegs;
    ba.steps = b->steps_dev;
    ba.steps_per_epoch = 0;      // segments index the table directly
    ba.table_epochs = 1;
    ba.cursor = b->cursor;
    HIP_TRY(gmf::launch_batch(b->prec, b->KP, ba, l.grid, b->st, l.updates_only));
  }
  return GMF_OK;
}

// Refill the step table with the next `ne` epochs of every fit (from each
// fit's current step counter) and reset the cursor.  Waits for the batch
// stream first: the previous table may still be read.
int refill_batch_table(Batch* b, int ne) {
  HIP_TRY(hipStreamSynchronize(b->st));
  b->host_steps.resize((size_t)b->table_epochs * b->steps_per_epoch);
  for (int e = 0; e < ne; ++e)
    for (size_t f = 0; f < b->fits.size(); ++f) {
      const Ctx* c = b->fits[f];
      const int rs = c->P.R * c->P.S;
      for (int k = 0; k < rs; ++k)
        b->host_steps[(size_t)e * b->steps_per_epoch + b->step_off[f] + k] =
            make_step(c, c->t + (int64_t)e * rs + k + 1);
    }
  HIP_TRY(hipMemcpyAsync(b->steps_dev, b->host_steps.data(),
                         sizeof(gmf::LevelStep) * (size_t)ne * b->steps_per_epoch,
                         hipMemcpyHostToDevice, b->st));
  HIP_TRY(gmf::launch_fill_i32(b->cursor, 1, 0, b->st));
  HIP_TRY(hipStreamSynchronize(b->st));
  b->used = 0;
  b->valid = ne;
  return GMF_OK;
}

void destroy_batch(Batch* b) {
  if (!b) return;
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  if (b->ev) (void)hipEventDestroy(b->ev);
  if (b->st) (void)hipStreamDestroy(b->st);
  delete b;
}

}  // namespace

extern "C" size_t gmf_batch_workspace_bytes(void* const* ctxs, int32_t nfits, int32_t table_epochs) {
  BatchSizes z;
  return batch_sizes(ctxs, nfits, table_epochs, z) ? z.total : 0;
}

extern "C" int gmf_batch_init(void** batch_out, void* const* ctxs, int32_t nfits, void* ws,
                              size_t ws_bytes, int32_t table_epochs, int32_t use_graph) {
  if (!batch_out) return fail(GMF_EINVAL, "batch_out is NULL");
  *batch_out = nullptr;
  BatchSizes z;
  if (!batch_sizes(ctxs, nfits, table_epochs, z))
    return fail(GMF_EINVAL, "need nfits >= 1 non-NULL contexts and table_epochs >= 1");
  if (!ws || (reinterpret_cast<uintptr_t>(ws) & 255) != 0 || ws_bytes < z.total)
    return fail(GMF_EWORKSPACE, "batch workspace NULL, misaligned or smaller than " +
                                    std::to_string(z.total) + " bytes");
  const Plan& P0 = as_ctx(ctxs[0])->P;
  for (int f = 0; f < nfits; ++f) {
    const Plan& P = as_ctx(ctxs[f])->P;
    if (P.prec != P0.prec || P.KP != P0.KP)
      return fail(GMF_EINVAL, "batched fits need one precision and one panel stride "
                              "(set gmf_config.panel_stride)");
    if (as_ctx(ctxs[f])->cfg.estimate_phi || as_ctx(ctxs[f])->cfg.estimate_alpha)
      return fail(GMF_EINVAL, "fits that estimate the dispersion or the NB shape run on their own");
    for (int g = 0; g < f; ++g)
      if (ctxs[g] == ctxs[f]) return fail(GMF_EINVAL, "a context appears twice in the batch");
  }
  Batch* b = new Batch();
  b->prec = P0.prec;
  b->KP = P0.KP;
  b->table_epochs = table_epochs;
  b->steps_per_epoch = z.steps_per_epoch;
  b->L = z.L;
  char* W = static_cast<char*>(ws);
  b->fits_dev = reinterpret_cast<gmf::LevelArgs*>(W + z.o_fits);
  b->segs_dev = reinterpret_cast<gmf::BatchSeg*>(W + z.o_segs);
  b->steps_dev = reinterpret_cast<gmf::LevelStep*>(W + z.o_steps);
  b->cursor = reinterpret_cast<int*>(W + z.o_cursor);
  b->scal = reinterpret_cast<double*>(W + z.o_scal);
  auto bail = [&](int code, const std::string& msg) {
    destroy_batch(b);
    return fail(code, msg);
  };
  if (hipStreamCreateWithFlags(&b->st, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&b->ev, hipEventDisableTiming) != hipSuccess)
    return bail(GMF_EDEVICE, "cannot create the batch stream");
  // descriptors and the static segment lists
  std::vector<gmf::LevelArgs> fa(nfits);
  int64_t off = 0;
  for (int f = 0; f < nfits; ++f) {
    Ctx* c = as_ctx(ctxs[f]);
    b->fits.push_back(c);
    fa[f] = level_args(c);
    fa[f].trace = nullptr;
    fa[f].trace_cap = 0;
    // In a batch the other fits supply the parallelism: one chunk of rows or
    // columns per update workgroup (no chunks run one after another); the
    // chunks and their sums are the same, so the results are too.
    {
      const Plan& P = c->P;
      int per = 1;
      for (int r = 0; r < P.R; ++r)
        for (int s = 0; s < P.S; ++s)
          per = std::max(per, upd_workgroups(P.nrows[r], P.mcols[s], P.row_chunk, P.col_chunk, 1));
      fa[f].upd_sub = 1;
      fa[f].upd_per_step = per;
      b->tile_wgs.push_back(P.rr_max * P.ct_max);
      b->upd_wgs.push_back(per);
    }
    b->step_off.push_back(off);
    off += (int64_t)c->P.R * c->P.S;
  }
  std::vector<gmf::BatchSeg> segs;
  for (int k = 0; k < b->L; ++k)
    for (int kind = 0; kind < 2; ++kind) {
      BatchLaunch l{(int)segs.size(), 0, 0, kind == 1};
      for (int f = 0; f < nfits; ++f) {
        const Plan& P = b->fits[f]->P;
        if (k >= P.R * P.S) continue;
        const int wgs = kind == 0 ? P.rr_max * P.ct_max : fa[f].upd_per_step;
        segs.push_back(gmf::BatchSeg{l.grid, f, kind, (int)(b->step_off[f] + k)});
        l.grid += wgs;
        ++l.nsegs;
      }
      if (l.nsegs > 0) b->launches.push_back(l);
    }
  if (hipMemcpyAsync(b->fits_dev, fa.data(), sizeof(gmf::LevelArgs) * fa.size(),
                     hipMemcpyHostToDevice, b->st) != hipSuccess ||
      hipMemcpyAsync(b->segs_dev, segs.data(), sizeof(gmf::BatchSeg) * segs.size(),
                     hipMemcpyHostToDevice, b->st) != hipSuccess ||
      hipStreamSynchronize(b->st) != hipSuccess)
    return bail(GMF_EDEVICE, "cannot upload the batch tables");
  if (use_graph < 0 || use_graph > 2) return bail(GMF_EINVAL, "mode must be 0, 1 or 2");
  b->mode = use_graph;
  if (use_graph == 1) {
    b->use_graph = true;
    if (hipStreamBeginCapture(b->st, hipStreamCaptureModeThreadLocal) != hipSuccess)
      return bail(GMF_EDEVICE, "cannot capture the batch epoch");
    const int rc = enqueue_batch_epoch(b);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(b->st, &g);
    b->graph = g;
    if (rc != GMF_OK || e != hipSuccess) return bail(GMF_EDEVICE, "batch epoch capture failed");
    if (hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0) != hipSuccess)
      return bail(GMF_EDEVICE, "cannot instantiate the batch epoch graph");
  }
  *batch_out = b;
  return GMF_OK;
}

extern "C" int gmf_batch_run(void* batch, int32_t epochs, int32_t eval_every,
                             double* dev_trace_host) {
  if (!batch) return fail(GMF_EINVAL, "batch is NULL");
  if (epochs < 0 || eval_every < 1) return fail(GMF_EINVAL, "bad epochs / eval_every");
  Batch* b = static_cast<Batch*>(batch);
  const int nfits = (int)b->fits.size();
  const int nevals = epochs / eval_every;
  // order after the work already queued on the fits' own streams
  for (Ctx* c : b->fits) {
    HIP_TRY(hipEventRecord(b->ev, c->st));
    HIP_TRY(hipStreamWaitEvent(b->st, b->ev, 0));
  }
  // a fresh table at every call: the fits may have been stepped on their own
  b->used = b->valid = 0;
  int ev_i = 0;
  auto evaluate = [&]() -> int {
    for (int f = 0; f < nfits; ++f) {
      Ctx* c = b->fits[f];
      gmf::DevArgs da = dev_args(c);
      HIP_TRY(gmf::launch_deviance(c->P.fam, c->P.KP, da, b->st));
      HIP_TRY(gmf::launch_finalize(da.partial, c->P.dev_tiles, nullptr, 0, c->at<int>(c->P.o_flag),
                                   b->scal + 8 * f, b->st));
    }
    std::vector<double> h(8 * (size_t)nfits);
    HIP_TRY(hipMemcpyAsync(h.data(), b->scal, sizeof(double) * h.size(), hipMemcpyDeviceToHost, b->st));
    HIP_TRY(hipStreamSynchronize(b->st));
    for (int f = 0; f < nfits; ++f) {
      dev_trace_host[(size_t)f * nevals + ev_i] = h[8 * f] + 2.0 * b->fits[f]->ktotal;
      if (h[8 * f + 5] != 0.0) {
        const int rc = check_flag(b->fits[f]);
        if (rc != GMF_OK) return rc;
      }
    }
    ++ev_i;
    return GMF_OK;
  };
  if (b->mode == 2) {
    for (int e = 0; e < epochs;) {
      int ne = std::min(b->table_epochs, epochs - e);
      if (dev_trace_host) ne = std::min(ne, eval_every - e % eval_every);
      int rc = refill_batch_table(b, ne);
      if (rc != GMF_OK) return rc;
      rc = enqueue_batch_leveled(b, ne);
      if (rc != GMF_OK) return rc;
      for (Ctx* c : b->fits) {
        c->t += (int64_t)ne * c->P.R * c->P.S;
        c->batched_upto = c->t;
      }
      e += ne;
      if (dev_trace_host && e % eval_every == 0) {
        rc = evaluate();
        if (rc != GMF_OK) return rc;
      }
    }
    HIP_TRY(hipEventRecord(b->ev, b->st));
    for (Ctx* c : b->fits) HIP_TRY(hipStreamWaitEvent(c->st, b->ev, 0));
    return GMF_OK;
  }
  for (int e = 0; e < epochs; ++e) {
    if (b->used == b->valid) {
      const int rc = refill_batch_table(b, std::min(b->table_epochs, epochs - e));
      if (rc != GMF_OK) return rc;
    }
    if (b->use_graph) {
      HIP_TRY(hipGraphLaunch(b->exec, b->st));
    } else {
      const int rc = enqueue_batch_epoch(b);
      if (rc != GMF_OK) return rc;
    }
    ++b->used;
    for (Ctx* c : b->fits) {
      c->t += (int64_t)c->P.R * c->P.S;
      c->batched_upto = c->t;
    }
    if ((e + 1) % eval_every == 0 && dev_trace_host) {
      const int rc = evaluate();
      if (rc != GMF_OK) return rc;
    }
  }
  // the fits' own streams continue after the batch
  HIP_TRY(hipEventRecord(b->ev, b->st));
  for (Ctx* c : b->fits) HIP_TRY(hipStreamWaitEvent(c->st, b->ev, 0));
  return GMF_OK;
}

extern "C" void gmf_batch_destroy(void* batch) {
  if (!batch) return;
  Batch* b = static_cast<Batch*>(batch);
  (void)hipStreamSynchronize(b->st);
  destroy_batch(b);
}

// ------------------------------------------------------------------ tuning --
extern "C" int gmf_tune(const gmf_config* cfg, void* ws, size_t ws_bytes, void* stream,
                        const void* Y, int32_t y_dtype, const float* X, const float* Z,
                        const float* W, const float* B0, const float* A0, const float* U0,
                        const float* V0, const int32_t* candidates, int32_t ncand, int32_t steps,
                        int32_t* best_host, double* us_per_step_host) {
  const std::string bad = check_config(cfg);
  if (!bad.empty()) return fail(GMF_EINVAL, "invalid config: " + bad);
  if (!candidates || ncand < 1 || steps < 1) return fail(GMF_EINVAL, "need candidates and steps >= 1");
  for (int i = 0; i < ncand; ++i) {
    gmf_config ci = *cfg;
    ci.tile_rows = candidates[i];
    if (!check_config(&ci).empty()) return fail(GMF_EINVAL, "bad candidate tile_rows");
    if (gmf_workspace_bytes(&ci, W != nullptr) > ws_bytes)
      return fail(GMF_EWORKSPACE, "tuning workspace smaller than a candidate needs");
  }
  hipStream_t st = static_cast<hipStream_t>(stream);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  int best = 0;
  double best_us = 0.0;
  int rc = GMF_OK;
  for (int i = 0; i < ncand && rc == GMF_OK; ++i) {
    gmf_config ci = *cfg;
    ci.tile_rows = candidates[i];
    void* ctx = nullptr;
    rc = gmf_init(&ctx, &ci, ws, ws_bytes, stream, Y, y_dtype, X, Z, W, B0, A0, U0, V0);
    if (rc != GMF_OK) break;
    Ctx* c = as_ctx(ctx);
    const int64_t warm = std::min<int64_t>(steps, (int64_t)c->P.R * c->P.S);
    rc = enqueue_steps(c, warm);
    if (rc == GMF_OK && hipEventRecord(e0, st) != hipSuccess) rc = fail(GMF_EDEVICE, "event");
    if (rc == GMF_OK) rc = enqueue_steps(c, steps);
    if (rc == GMF_OK && (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess))
      rc = fail(GMF_EDEVICE, "event");
    float ms = 0.f;
    if (rc == GMF_OK && hipEventElapsedTime(&ms, e0, e1) != hipSuccess) rc = fail(GMF_EDEVICE, "event");
    if (rc == GMF_OK) rc = check_flag(c);
    gmf_destroy(ctx);
    if (rc != GMF_OK) break;
    const double us = 1e3 * ms / steps;
    if (us_per_step_host) us_per_step_host[i] = us;
    if (i == 0 || us < best_us) {
      best_us = us;
      best = candidates[i];
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc != GMF_OK) return rc;
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune[tune_key(cfg)] = TuneVal{best, best_us};
  }
  if (best_host) *best_host = best;
  return GMF_OK;
}

extern "C" int32_t gmf_tune_lookup(const gmf_config* cfg) {
  if (!cfg || !check_config(cfg).empty()) return 0;
  return tune_lookup(cfg);
}

extern "C" void gmf_tune_table_clear(void) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tune.clear();
}

extern "C" int gmf_tune_table_save(const char* path) {
  if (!path) return fail(GMF_EINVAL, "path is NULL");
  std::ofstream out(path);
  if (!out) return fail(GMF_EINVAL, std::string("cannot write ") + path);
  out << "# libgmf tile-rows table: precision family panel_stride log2|I| log2|J| tile_rows us_per_step\n";
  std::lock_guard<std::mutex> lk(g_tune_mu);
  for (const auto& kv : g_tune)
    out << kv.first.prec << ' ' << kv.first.fam << ' ' << kv.first.KP << ' ' << kv.first.nb_log2 << ' '
        << kv.first.mb_log2 << ' ' << kv.second.tile_rows << ' ' << kv.second.us_per_step << '\n';
  return out.good() ? GMF_OK : fail(GMF_EINVAL, std::string("write failed: ") + path);
}

extern "C" int gmf_tune_table_load(const char* path) {
  if (!path) return fail(GMF_EINVAL, "path is NULL");
  std::ifstream in(path);
  if (!in) return fail(GMF_EINVAL, std::string("cannot read ") + path);
  std::map<TuneKey, TuneVal> rows;
  std::string line;
  int lineno = 0;
  while (std::getline(in, line)) {
    ++lineno;
    if (line.empty() || line[0] == '#') continue;
    std::istringstream ls(line);
    TuneKey k;
    TuneVal v;
    if (!(ls >> k.prec >> k.fam >> k.KP >> k.nb_log2 >> k.mb_log2 >> v.tile_rows >> v.us_per_step) ||
        v.tile_rows < 32 || v.tile_rows % 32 != 0 || v.tile_rows > 4096)
      return fail(GMF_EINVAL, std::string(path) + ": bad line " + std::to_string(lineno));
    rows[k] = v;
  }
  std::lock_guard<std::mutex> lk(g_tune_mu);
  for (const auto& kv : rows) g_tune[kv.first] = kv.second;
  return GMF_OK;
}
