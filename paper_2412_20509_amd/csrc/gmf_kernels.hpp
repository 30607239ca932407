// Internal declarations shared by the HIP kernels and the host side of libgmf.
// Device code targets gfx950 (CDNA4): 64-lane wavefronts, MFMA 16x16 tiles.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gmf {

// ---------------------------------------------------------------- geometry --
// A step tile is processed by one workgroup of 4 wavefronts.  The workgroup
// owns a range of `rows_per_wg` block rows (walked in groups of 32) and a
// strip of 128 block columns; wavefront w owns columns [32w, 32w+32) of the
// strip.  Every 32x32 piece is four 16x16 MFMA output tiles.
constexpr int kWave = 64;
constexpr int kTileWaves = 4;
constexpr int kTileThreads = kWave * kTileWaves;
constexpr int kWaveCols = 32;
constexpr int kTileCols = kWaveCols * kTileWaves;
constexpr int kRowGroup = 32;

// Four counts as float32: from a float4 of the float32 layout or from the four
// 16-bit integers (uint2) of the compact one (exact: every count <= 65535).
__device__ __forceinline__ float4 counts_f4(const float4& y) { return y; }
__device__ __forceinline__ float4 counts_f4(const uint2& u) {
  return make_float4((float)(u.x & 0xffffu), (float)(u.x >> 16), (float)(u.y & 0xffffu),
                     (float)(u.y >> 16));
}

// Workgroups of a launch are dealt to the eight XCDs in turn (workgroup b to
// XCD b mod 8), each XCD with its own L2.  xcd_tile(b, n) renumbers the n
// tiles of a launch so that every XCD takes one contiguous range of them:
// XCD x takes tiles [x q + min(x, r), ..) with q = n / 8, r = n mod 8 (q + 1
// tiles when x < r), in dispatch order.  Tiles that share panel rows (the
// column strips of one row range) then run on one XCD and read those rows
// from its L2 once.  A bijection of [0, n) for every n.
constexpr int kXcds = 8;
__host__ __device__ inline int xcd_tile(int b, int n) {
  const int x = b % kXcds, k = b / kXcds;
  const int q = n / kXcds, r = n % kXcds;
  return x * q + (x < r ? x : r) + k;
}

// Kernel family selector: three fast paths (complete data, fixed dispersion)
// and kGeneric, whose epilogue switches at run time on FamilyArgs::code over
// the six families of Supplementary Table 1 (codes as GMF_POISSON ..
// GMF_INVGAUSS), imputes missing entries (NaN) by their mean and reads the
// NB shape per column and the estimated dispersion / NB shape when given.
enum Family { kPoisson = 0, kNegBin = 1, kGaussian = 2, kGeneric = 7 };
enum FamilyCode { kCodePoisson = 0, kCodeNegBin = 1, kCodeGaussian = 2, kCodeGamma = 3,
                  kCodeBernoulli = 4, kCodeInvGauss = 5 };
enum LinkCode { kLinkLog = 0, kLinkIdentity = 1, kLinkLogit = 2 };
// kBF16X3: bfloat16 MFMA on operands split into a high and a low bfloat16
// part (x = hi + lo), three products per contraction (hi*hi + hi*lo + lo*hi).
enum Prec { kF32 = 0, kBF16 = 1, kBF16X3 = 2 };

struct FamilyArgs {
  float phi_inv;       // 1 / phi
  float nb_alpha;      // NB shape
  float eta_lo;        // log(eps)   (log link)
  float eta_hi;        // eta_max    (log link; the logit link clamps to +-eta_max)
  int code, link;      // generic path: family and link codes
  const float* alpha_col;   // generic path: NB shape per permuted column, or null
  const double* est;        // generic path: [phi, alpha] in use (estimated), or null
};

// Starting values of projected rows (warm.hip).  Y: the caller's new rows in
// original order (n x m, int32 or float32); Prow: their panel (n x KP) with X
// filled (and Gamma for row_select); Pcol_orig: the frozen column panel in the
// caller's original column order (m x KP); Ucand: candidate scores (n x d) for
// row_select; dev_out (optional): per row [deviance with Ucand, with 0];
// fallback: count of rows that start from 0.  Requires p + q + d <= 64.
struct WarmArgs {
  const void* Y;
  int64_t n;
  int m, p, q, d, KP;
  float* Prow;
  const float* Pcol_orig;
  FamilyArgs f;
  const float* Ucand;
  double* dev_out;
  unsigned long long* fallback;
};

hipError_t launch_row_intercept(const WarmArgs& a, bool y_int, bool log_link, hipStream_t s);
hipError_t launch_row_select(const WarmArgs& a, int fam, bool y_int, hipStream_t s);

// One step handed to a level launch, with its block geometry.
struct LevelStep {
  int r, s;            // row block and column block
  int slot;            // partial-buffer slot
  int n_b, m_b;        // |I_r|, |J_s|
  int n_rr, n_ct, rpw; // tiling: row ranges, column strips, rows per range
  int ldy;             // padded row stride of the block
  int ro, co;          // first permuted row / column of the block
  int pad;
  int64_t yoff;        // offset of the block in the block-major Y
  double stepsize;     // rho_t * alpha_t
  int64_t t;           // global step number (from 1)
};

constexpr int kMaxLevelSteps = 32;   // tile steps + update steps per launch

struct LevelArgs {
  // data in the workspace (permuted, block-major)
  const float* Y; const float* W;
  const uint16_t* Yc;  // the counts as 16-bit integers (same layout), or null: read Y
  float* Prow; float* Pcol;
  double* Grow; double* Hrow; double* Gcol; double* Hcol;
  int64_t LDtot;
  // per row block r / column block s geometry
  const int* ro; const int* nrows; const int* rpw; const int* nrr;
  const int* co; const int* mcols; const int* ldy; const int* nct; const int64_t* coP;
  int rr_max, ct_max;
  int64_t n, m;
  // partial slots
  float* Upart; float* Vpart; double* devpart;
  int64_t slot_u_elems, slot_v_elems, slot_dev_elems;
  // update work split
  // update work split: an update workgroup walks upd_sub chunks of row_chunk
  // rows (or col_chunk columns); upd_per_step workgroups cover a step
  int row_chunk, col_chunk, upd_sub, upd_per_step;
  // numerics
  FamilyArgs f;
  int fam;             // family (read by the batched kernel; the others take it as a template)
  int p, q, d, KU, KV, KP;
  double lam_B, lam_A, lam_U, lam_V;
  double a1, a2, damping;
  double* devring; int devring_len;
  int* err_flag;
  // optional per-workgroup trace: 8 x u64 per workgroup (see gmf_set_trace)
  unsigned long long* trace; long long trace_cap; unsigned long long trace_base;
  unsigned long long launch_id;
  // the steps of this launch: [0, n_tile_steps) run tiles, the next
  // n_upd_steps run their updates
  int n_tile_steps, n_upd_steps;
  LevelStep steps[kMaxLevelSteps];
};

// Batched level launches over many fits.  A launch runs one phase (tiles or
// updates) of one step of several fits; its workgroups are cut into segments,
// one per (fit, step), in ascending `start` order.  The steps come from a
// device table of `table_epochs` epochs x `steps_per_epoch` entries (every
// fit's steps of one epoch, fit f at its own offset); *cursor selects the
// epoch (mod table_epochs), so one recorded launch sequence serves every
// epoch.
struct BatchSeg {
  int start;        // first workgroup of the segment
  int fit;          // index into fits
  int kind;         // 0: tiles, 1: updates
  int step_index;   // entry inside an epoch of the step table
};
struct BatchArgs {
  const LevelArgs* fits;
  const BatchSeg* segs;
  int nsegs;
  const LevelStep* steps;
  int64_t steps_per_epoch;
  int table_epochs;
  const int* cursor;
};

// updates_only: every segment of the launch is an update segment (kind 1);
// they then run in a kernel with only the update tasks' LDS.
hipError_t launch_batch(int prec, int KP, const BatchArgs& a, int grid, hipStream_t s,
                        bool updates_only = false);
hipError_t launch_advance_cursor(int* cursor, hipStream_t s);

// nw: wavefronts per tile workgroup, 4 or 8 (level_supports_nw8).
// ev_start / ev_stop (optional): HIP events stamped at the start and end of
// this kernel's execution.
hipError_t launch_level(int prec, int fam, int KP, bool want_dev, int nw, const LevelArgs& a,
                        int grid, hipStream_t s, hipEvent_t ev_start = nullptr,
                        hipEvent_t ev_stop = nullptr);
bool level_supports_nw8(int prec, int KP);

// One row-only step of the projection (project.hip): column block J_s of the
// new rows.  Y: the block's counts (n rows, stride ldy, m_b columns; columns
// m_b .. ldy-1 are zero); Prow: the new rows' panel (n x KP, updated in place);
// Pcol: the block's frozen column panel rows (m_b x KP); Grow, Hrow: the rows'
// EMAs (n x KU, KU = q + d); scale_m = m / m_b; stepsize = rho_t alpha_t.
struct ProjStepArgs {
  const float* Y;
  const uint16_t* Yc;   // the same counts as 16-bit integers, or null: read Y
  int ldy, m_b;
  float* Prow;
  const float* Pcol;
  double* Grow; double* Hrow;
  int64_t n;
  int p, q, KU;
  double scale_m, lam_A, lam_U, a1, a2, damping, stepsize;
  FamilyArgs f;
  int* err_flag;
};
hipError_t launch_project_step(int prec, int fam, int KP, const ProjStepArgs& a, hipStream_t s);

struct DevArgs {
  const float* Y; const float* W;
  const uint16_t* Yc;          // 16-bit copy of the counts, or null: read Y
  const float* Prow; const float* Pcol;
  const int* tile_block;       // tile -> block id
  const int* tile_first;       // block id -> first tile id
  const int64_t* blk_yoff;     // block id -> Y offset
  const int* blk_row0; const int* blk_col0;
  const int* blk_nb; const int* blk_mb; const int* blk_ldy;
  const int* blk_rpw; const int* blk_nct;
  FamilyArgs f;
  double* partial;             // one per tile
  int n_tiles;
  int grid_cap;                // deviance: at most this many workgroups (0 = one per tile)
};
hipError_t launch_deviance(int fam, int KP, const DevArgs& a, hipStream_t s);
// Yc[i] = Yb[i] for the count elements of the block-major layout; sets
// *flag = 1 if any of them is not an integer in [0, 65535] (then Yc is not
// to be used).
hipError_t launch_compact_counts(const float* Yb, int64_t count, uint16_t* Yc, int* flag,
                                 hipStream_t s);

// Per-row deviance (aux.hip).  Yb, Wb: block-major counts and weights (Wb may
// be null); rowblk, rowloc: caller row i -> row block and row inside it; ro:
// first permuted row of each row block; nrows: rows per row block; rowbase:
// offset of each row block in Yb; co, mcols, coloff, ld: first permuted
// column, width, padded offset and row stride of each column block; out: n
// doubles in the caller's row order.
struct RowDevArgs {
  const float* Yb; const float* Wb;
  const float* Prow; const float* Pcol;
  const int* rowblk; const int* rowloc; const int* ro; const int* nrows;
  const int64_t* rowbase;
  const int* co; const int* mcols; const int64_t* coloff; const int* ld;
  int64_t n;
  int S;
  FamilyArgs f;
  double* out;
};
hipError_t launch_row_deviance(int fam, int KP, const RowDevArgs& a, hipStream_t s);
// a.partial[tile] = sum over the tile of w c(y), the count-only part of half
// the unit deviance (float64; nothing for the Gaussian family).
hipError_t launch_count_sum(int fam, const DevArgs& a, hipStream_t s);
hipError_t launch_sum_partials(const double* partial, int count, double* out,
                               hipStream_t s);
hipError_t launch_norms(const float* Prow, const float* Pcol, int KP, int64_t n, int64_t m,
                        int p, int q, int d, double* partial, int nblocks, hipStream_t s);
// out[0] = sum of dev, out[1..4] = the four norm sums (0 without norm),
// out[5] = *flag (0 without flag).
hipError_t launch_finalize(const double* dev, int ndev, const double* norm, int nnorm,
                           const int* flag, double* out, hipStream_t s);

// Init / copy-out kernels.
hipError_t launch_permute_y(const void* Y, int y_is_int, const float* W, int64_t n,
                            int64_t m, const int* row_block, const int* row_local,
                            const int* col_block, const int* col_local,
                            const int64_t* blk_row_base, const int* blk_nrows,
                            const int64_t* blk_col_off, const int* blk_ld, float* Yb,
                            float* Wb, int* err_flag, hipStream_t s, int allow_missing = 0,
                            int check = 0);
hipError_t launch_pack_panel(const float* M0, int c0, const float* M1, int c1,
                             const float* M2, int c2, const int* perm, int64_t rows,
                             int KP, float* P, hipStream_t s);
hipError_t launch_unpack_panel(const float* P, int KP, const int* perm, int64_t rows,
                               int col0, int ncols, float* out, hipStream_t s);
hipError_t launch_unpack_moments(const double* M, int K, const int* perm,
                                 int64_t rows, double* out, hipStream_t s);
hipError_t launch_fill_f64(double* p, int64_t count, double v, hipStream_t s);
hipError_t launch_fill_i32(int* p, int64_t count, int v, hipStream_t s);
hipError_t launch_iota(int* p, int64_t count, hipStream_t s);
hipError_t launch_sumsq(const float* P, int KP, int64_t rows, int col0, int ncols,
                        double* partial, int nblocks, hipStream_t s);

// Parameter initialization (init.hip).  A pass computes each entry of one of
// mode 0: L = g(y + c_off); 1: L - eta; 2: Pearson residual; 3: deviance
// residual; 4: 1 for an observed entry (eta over the first ke panel columns,
// mu clamped as in the fit)
// and contracts it with the dense operand Q (kq <= 64 columns, permuted
// order): the row pass writes part[s][i][:] = sum_{j in J_s} E_ij Q[j][:] for
// every column block s (grid: row tiles x S); the column pass writes
// part[c][j][:] = sum_{i in chunk c} E_ij Q[i][:] for every row chunk c
// (grid: column tiles x chunks).  nout: rows of one partial set (n or m).
struct InitPassArgs {
  const float* Yb; const float* Wb;
  int64_t LDtot;
  const float* Prow; const float* Pcol;
  int KP, ke;
  const int* ro; const int* nrows; const int* co; const int* mcols; const int* ldy;
  const int64_t* coP;
  int mode, fam, log_link;
  float c_off;
  FamilyArgs f;
  const float* colfill;   // mode 0: per permuted column, the value of missing entries (or null)
  const float* Q;
  int kq;
  float* part;
  int64_t nout;
  const int* tiles;       // (block, first local row/column) per workgroup x
  const int* chunks;      // column pass: (row block, first local row, rows) per workgroup y
};
hipError_t launch_init_pass(const InitPassArgs& a, bool row_pass, int grid_x, int grid_y,
                            hipStream_t st);
hipError_t launch_sum_parts(const float* part, int nparts, int64_t stride, int64_t count,
                            double* out64, float* out32, hipStream_t st);
hipError_t launch_gram(const double* A, int64_t rows, int k, double* part, int nparts, double* out,
                       hipStream_t st);
hipError_t launch_apply(const double* A, int64_t rows, int ka, int kb, const double* M,
                        const double* scale, double* out64, float* out32, float* panel, int KP,
                        int col0, hipStream_t st);
hipError_t launch_panel_cols(float* P, int KP, int64_t rows, int col0, int ncols, double* out64,
                             float* out32, int zero, hipStream_t st);
hipError_t launch_ratio(const double* num, const double* den, int64_t count, float* out,
                        hipStream_t st);

// Stochastic dispersion / NB-shape estimation (Appendix B, aux.hip).
// block_stats: per workgroup of 16 block rows, float64 sums over the observed
// entries of the block of w (y - mu)^2 / nu(mu), w mu^2 and
// w ((y - mu)^2 - mu) at the current (pre-step) parameters -> partial[3 wg +
// 0..2].  est_update: sums the partials in order, phi^ = scale_phi * S0,
// alpha^ = S1 / S2, and smooths est[0] (phi) and est[1] (alpha) with weight
// rho (alpha^ floored at eps).
struct BlockStatsArgs {
  const float* Y; const float* W;   // the block (row stride ldy)
  const float* Prow; const float* Pcol;   // the block's panel rows (stride KP)
  int ldy, n_b, m_b, KP;
  int64_t col0;                     // first permuted column of the block
  FamilyArgs f;
  double* partial;
};
hipError_t launch_block_stats(const BlockStatsArgs& a, hipStream_t s);
int block_stats_workgroups(int n_b);
hipError_t launch_est_update(const double* partial, int nwg, double* est, double scale_phi,
                             double rho, double eps, int est_phi, int est_alpha, hipStream_t s);

// Held-out reconstruction error (Section 5.2).  observed_sum: per deviance
// tile, the sum and the count of the observed (non-NaN) training entries ->
// partial[2 tile + 0..1].  heldout: per workgroup of 16 permuted rows, over
// the entries that Ytest (caller order, n x m) holds a value for (an int32
// >= 0 or a finite float32; negative ints and NaN mark the other entries):
// float64 sums of [log((1+y)/(1+mu))]^2, [log((1+y)/(1+ybar))]^2, the Poisson
// deviances D(y, mu), D(y, ybar), the family's deviances D(y, mu), D(y, ybar)
// and the count -> partial[8 wg + 0..6].
hipError_t launch_observed_sum(const DevArgs& a, double* partial, hipStream_t s);
struct HeldoutArgs {
  const void* Ytest; int y_int;
  const float* Prow; const float* Pcol; int KP;
  const int* row_perm; const int* col_perm;   // permuted -> caller index
  int64_t n, m;
  double ybar;
  FamilyArgs f;
  double* partial;
};
hipError_t launch_heldout(const HeldoutArgs& a, hipStream_t s);
// Sets bit 2 of *err_flag if an entry is not a positive finite number.
hipError_t launch_check_positive(const float* x, int64_t count, int* err_flag, hipStream_t s);
int heldout_workgroups(int64_t n);

// Identifiability post-processing (float64).
struct PostArgs {
  const float* Prow; const float* Pcol;   // current iterate (permuted order)
  int64_t n, m; int p, q, d, KP;
  const int* row_perm; const int* col_perm;   // permuted -> original index
  double* gram_part;   // scratch: per-block partial Gram matrices
  double* small;       // scratch: small matrices (see post.hip)
  int* first_nz;       // unused (keys live after the small matrices)
  int* err_flag;       // bit 4 set if a covariate Gram is not positive definite
  float* B; float* A; float* U; float* V;     // outputs, original order
  int nblocks_row, nblocks_col;
};
hipError_t launch_postprocess(const PostArgs& a, hipStream_t s);
size_t postprocess_scratch_doubles(int64_t n, int64_t m, int KP, int nblocks);

}  // namespace gmf
