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

enum Family { kPoisson = 0, kNegBin = 1, kGaussian = 2 };
enum Prec { kF32 = 0, kBF16 = 1 };

// One block B = I_r x J_s as seen by the tile kernels.
struct BlockView {
  const float* Y;      // block base; element (i, j) at Y[i * ldy + j]
  const float* W;      // same layout, or nullptr for unit weights
  const float* Prow;   // [X | Gamma | U | 0] rows of I_r, row stride KP
  const float* Pcol;   // [B | Z | V | 0] rows of J_s, row stride KP
  int64_t ldy;         // padded row stride (multiple of 4)
  int n_b, m_b;        // |I_r|, |J_s|
  int rows_per_wg;     // multiple of kRowGroup
  int n_rr, n_ct;      // row ranges and column strips of the tiling
};

struct FamilyArgs {
  float phi_inv;       // 1 / phi
  float nb_alpha;      // NB shape
  float eta_lo;        // log(eps)   (log link)
  float eta_hi;        // eta_max    (log link)
};

struct TileArgs {
  BlockView b;
  FamilyArgs f;
  float* Upart;        // [n_ct][n_b][2*KU] : column-strip partial sums, G then H
  float* Vpart;        // [n_rr][m_b][2*KV] : row-range partial sums, G then H
  double* devpart;     // [n_rr * n_ct]     : per-tile deviance partial sums
  int p, q, d, KU, KV;
  int want_dev;
};

struct UpdateArgs {
  float* Prow;         // rows of I_r in the row panel (stride KP)
  float* Pcol;         // rows of J_s in the column panel (stride KP)
  double* Grow; double* Hrow;   // moments of [Gamma, U] for I_r (stride KU)
  double* Gcol; double* Hcol;   // moments of [B, V] for J_s (stride KV)
  const float* Upart; const float* Vpart; const double* devpart;
  int n_b, m_b, n_ct, n_rr, n_tiles;
  int p, q, d, KU, KV, KP;
  double scale_m, scale_n;      // m / |J_s|, n / |I_r|
  double lam_B, lam_A, lam_U, lam_V;
  double a1, a2, stepsize, damping;
  double* dev_out;              // where the block deviance of this step goes
  int* err_flag;                // set to 1 on a non-finite parameter
  int want_dev;
};

// ------------------------------------------------------------ launchers ----
// Host-side launchers implemented in the .hip files.
hipError_t launch_tile(int prec, int fam, int KP, const TileArgs& a, hipStream_t s);
hipError_t launch_update(const UpdateArgs& a, hipStream_t s);

struct DevArgs {
  const float* Y; const float* W;
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
};
hipError_t launch_deviance(int fam, int KP, const DevArgs& a, hipStream_t s);
hipError_t launch_sum_partials(const double* partial, int count, double* out,
                               hipStream_t s);

// Init / copy-out kernels.
hipError_t launch_permute_y(const void* Y, int y_is_int, const float* W, int64_t n,
                            int64_t m, const int* row_block, const int* row_local,
                            const int* col_block, const int* col_local,
                            const int64_t* blk_row_base, const int* blk_nrows,
                            const int64_t* blk_col_off, const int* blk_ld, float* Yb,
                            float* Wb, int* err_flag, hipStream_t s);
hipError_t launch_pack_panel(const float* M0, int c0, const float* M1, int c1,
                             const float* M2, int c2, const int* perm, int64_t rows,
                             int KP, float* P, hipStream_t s);
hipError_t launch_unpack_panel(const float* P, int KP, const int* perm, int64_t rows,
                               int col0, int ncols, float* out, hipStream_t s);
hipError_t launch_unpack_moments(const double* M, int K, const int* perm,
                                 int64_t rows, double* out, hipStream_t s);
hipError_t launch_fill_f64(double* p, int64_t count, double v, hipStream_t s);
hipError_t launch_fill_i32(int* p, int64_t count, int v, hipStream_t s);
hipError_t launch_sumsq(const float* P, int KP, int64_t rows, int col0, int ncols,
                        double* partial, int nblocks, hipStream_t s);

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
