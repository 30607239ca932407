/*
 * gmf.h -- C ABI of libgmf: block-wise adaptive SGD for generalized matrix
 * factorization (GMF) on one AMD Instinct MI355X (gfx950).
 *
 * Model (Section 2, eq. 1-3).  Y is an n x m matrix whose entries follow an
 * exponential dispersion family with mean mu_ij and
 *     g(mu_ij) = eta_ij = x_i' beta_j + gamma_i' z_j + u_i' v_j,
 * i.e. eta = X B' + Gamma Z' + U V' with X n x p, B m x p, Gamma n x q,
 * Z m x q, U n x d, V m x d.  The penalised negative log-likelihood of eq. 6
 * is minimised by the block-wise adaptive SGD of Algorithm 1, extended to the
 * covariate effects as in Appendix B.
 *
 * Conventions for every call:
 *   - Array arguments are DEVICE pointers unless the name ends in _host.
 *     Matrices are row-major, dense, in the caller's original row/column
 *     order, float32 unless stated.
 *   - The caller owns every buffer it passes.  The library keeps no pointer to
 *     a caller array after the call returns, except the workspace given to
 *     gmf_init, which must stay alive until gmf_destroy.
 *   - The library allocates no device memory: all device state lives in the
 *     caller's workspace (size from gmf_workspace_bytes).  It allocates a small
 *     host-side context object.
 *   - Work is enqueued on the caller's HIP stream; calls that return a *_host
 *     value synchronise that stream first.
 *   - Every call returns GMF_OK (0) or a negative code; gmf_last_error() gives
 *     a message for the calling thread.  A non-finite parameter produced by a
 *     step raises a device flag that the next synchronising call reports as
 *     GMF_ENUMERIC.
 *   - Calls on one context must not overlap (one stream, one thread at a time).
 */
#ifndef GMF_H_
#define GMF_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  GMF_OK = 0,
  GMF_EINVAL = -1,      /* bad argument, shape or configuration */
  GMF_EWORKSPACE = -2,  /* workspace NULL, misaligned or too small */
  GMF_EDEVICE = -3,     /* HIP runtime error or missing gfx950 device */
  GMF_ENUMERIC = -4,    /* a step produced a non-finite value */
  GMF_ENOTCONV = -5     /* gmf_fit stopped at max_epochs without meeting tol */
};

/* Families and links of Supplementary Table 1.  Pairs: Poisson, NB, Gamma and
 * inverse Gaussian with the log link, Gaussian with the identity link,
 * Bernoulli with the logit link.  Poisson, NB and Gaussian on complete data
 * with a fixed dispersion run specialised epilogues in every precision; the
 * other families, missing entries, per-column NB shapes and dispersion
 * estimation run a generic epilogue (family switched at run time) in FP32. */
enum { GMF_POISSON = 0, GMF_NEGBIN = 1, GMF_GAUSSIAN = 2, GMF_GAMMA = 3, GMF_BERNOULLI = 4,
       GMF_INVGAUSS = 5 };
enum { GMF_LINK_LOG = 0, GMF_LINK_IDENTITY = 1, GMF_LINK_LOGIT = 2 };
/* Arithmetic of the block contractions (eta and the four gradient sums).
 * FP32: float32 matrix-core products with float32 accumulation.
 * BF16: bfloat16 operands (round to nearest even), float32 accumulation.
 * BF16X3: bfloat16 matrix-core products on operands split into a high and a
 *   low bfloat16 part (x = hi + lo, lo = bf16(x - hi)), three products per
 *   contraction (lo*hi + hi*lo + hi*hi), float32 accumulation: about 16
 *   mantissa bits per operand instead of 8, in eta and in all four sums.
 * In all, the smoothed moments and the deviance sums are float64. */
enum { GMF_PREC_FP32 = 0, GMF_PREC_BF16 = 1, GMF_PREC_BF16X3 = 2 };
/* Element type of the Y array handed to gmf_init. */
enum { GMF_Y_INT32 = 0, GMF_Y_FLOAT32 = 1 };

typedef struct gmf_config {
  int32_t family;     /* GMF_POISSON, GMF_NEGBIN or GMF_GAUSSIAN             */
  int32_t link;       /* GMF_LINK_LOG (Poisson, NB) or GMF_LINK_IDENTITY     */
  int32_t precision;  /* GMF_PREC_FP32, GMF_PREC_BF16 or GMF_PREC_BF16X3     */
  int32_t bias_mode;  /* 0: alpha_t = (1-(1-a2)^t)/(1-(1-a1)^t) (Adam form);
                         1: alpha_t = (1-a2^t)/(1-a1^t) as printed (eq. 11)    */
  int64_t n, m;       /* rows and columns of Y                                 */
  int32_t d, p, q;    /* rank and covariate counts; p, q >= 0, 1 <= d,
                         p + q + d <= 64                                       */
  int32_t R, S;       /* number of row blocks and column blocks (Algorithm 1) */
  double phi;         /* dispersion (1 for Poisson and NB)                     */
  double nb_alpha;    /* NB shape alpha > 0: Var = mu + mu^2/alpha             */
  double lambda[4];   /* ridge weights for B, Gamma, U, V (eq. 6, Appendix B) */
  double rate0, decay, tau; /* rho_t = rate0 / (1 + rate0 decay t)^tau        */
  double alpha1, alpha2;    /* EMA weights of the new estimate (eq. 12)       */
  double damping;     /* delta added to the smoothed Hessian in the step      */
  double eps;         /* mu floor: eta is clamped to >= log(eps) (log link)   */
  double eta_max;     /* eta ceiling for the log link                         */
  uint64_t seed;      /* schedule seed: partitions and row-block draws        */
  int32_t tile_rows;  /* rows per step tile (multiple of 32), 0 = automatic   */
  int32_t skip_block_deviance; /* 1: steps do not form the block deviance   */
  int32_t panel_stride; /* floats per panel row: 0 = automatic (p+q+d rounded
                           up to 16; for BF16 and BF16X3 above 16 up to 32);
                           else 16, 32, 48 or 64 (BF16, BF16X3: 16, 32 or 64)
                           and >= p+q+d.  Fits run together by gmf_batch_*
                           must share it.  At stride 16 the bfloat16 products
                           are 16x16x16, above it 16x16x32.                    */
  int32_t tile_waves;   /* wavefronts per step tile: 4 (each takes 32 rows x 32
                           columns of a 32-row group) or 8 (16 rows x 32
                           columns each, half the per-wavefront work; FP32
                           stride 16/32, BF16 32 only); 0 = automatic: 4,
                           the faster one at every measured shape            */
  int32_t eval_overlap; /* gmf_run's deviance evaluations: 0 = on the
                           context's stream after the epoch's steps (full
                           grid); 1 = on a second stream from a copy of the
                           panels, overlapped with the following steps       */
  int32_t allow_missing; /* 1: a negative int32 or a NaN float32 in Y is a
                           missing entry, imputed by its current mean at every
                           step (y <- mu, Section 3.2.2: no gradient, its
                           Fisher weight kept, no deviance); the deviance
                           and its per-row form cover the observed entries  */
  int32_t estimate_phi;  /* 1: the dispersion phi (Gaussian, Gamma, inverse
                           Gaussian) is estimated during the fit by the
                           smoothed stochastic Pearson estimator of Appendix
                           B ("Unknown dispersion parameter"), starting at
                           cfg.phi                                           */
  int32_t estimate_alpha; /* 1: the NB shape is estimated during the fit by the
                           smoothed stochastic moment estimator of Appendix
                           B ("Negative Binomial inflation parameter"),
                           starting at cfg.nb_alpha, floored at cfg.eps.
                           With either estimator every step waits for the
                           previous one (its D1, D2 use the estimate it
                           updated): two launches per step               */
  int32_t compact_counts; /* 1 (default): for the Poisson and NB families on
                           their fixed-shape epilogue (no missing entries,
                           no estimation, no per-column shapes) with every
                           count in [0, 65535], the workspace also holds the
                           counts as 16-bit integers (2 B per entry more),
                           and the bfloat16 step tiles (BF16, BF16X3) and the
                           full deviance read those instead of the float32
                           copy: the same values, half the bytes, the same
                           results bit for bit.  Decided at gmf_init from
                           the data (gmf_compact_counts reports it); 0: the
                           float32 counts only                             */
} gmf_config;

/* Fill *cfg with the defaults: Poisson/log, FP32, n=m=0, d=1, p=q=0, R=10,
 * S=5, phi=1, nb_alpha=5, lambda=(0,0,1,1), rate0=0.05, decay=0.05,
 * tau=0.75, alpha1=0.1, alpha2=0.01, damping=1e-3, eps=1e-8, eta_max=30,
 * bias_mode=0, seed=0, tile_rows=0, skip_block_deviance=0, panel_stride=0,
 * tile_waves=0, eval_overlap=0, allow_missing=0, estimate_phi=0,
 * estimate_alpha=0, compact_counts=1. */
void gmf_config_default(gmf_config* cfg);

/* Device bytes gmf_init needs for cfg (with_weights != 0 when a weight
 * matrix will be passed).  Returns 0 for an invalid cfg. */
size_t gmf_workspace_bytes(const gmf_config* cfg, int32_t with_weights);

/* gmf_init -- set up a context: draw the partitions {I_r}, {J_s} once
 * (Algorithm 1, before the loop) from SplitMix64 stream 0/1 of cfg->seed with
 * Fisher-Yates shuffles, and copy Y, W, X, Z and the starting parameters into
 * the workspace, physically permuted so that every block I_r x J_s is a dense
 * rectangle.
 *   Y  n x m, GMF_Y_INT32 counts (0 <= y < 2^24) or GMF_Y_FLOAT32 reals;
 *      Poisson and NB need integer counts >= 0, Gamma and inverse Gaussian
 *      y > 0, Bernoulli y in {0, 1}; with cfg.allow_missing a negative int32
 *      or a NaN float32 marks a missing entry.
 *   X  n x p, Z m x q (may be NULL when p or q is 0).
 *   W  n x m positive weights w_ij of a_ij(phi) = phi/w_ij (eq. 2), or NULL
 *      for w = 1; non-NULL requires with_weights in gmf_workspace_bytes.
 *   B0 m x p, A0 n x q (Gamma), U0 n x d, V0 m x d starting values.
 *   stream: hipStream_t (NULL = default stream).
 * Synchronises the stream.  Errors: GMF_EINVAL (shapes, cfg, NULL arrays),
 * GMF_EWORKSPACE, GMF_EDEVICE. */
int gmf_init(void** ctx_out, const gmf_config* cfg, void* workspace,
             size_t ws_bytes, void* stream, const void* Y, int32_t y_dtype,
             const float* X, const float* Z, const float* W, const float* B0,
             const float* A0, const float* U0, const float* V0);

/* gmf_step -- run nsteps iterations of Algorithm 1 (steps 1-4) with the
 * covariate extension of Appendix B.  Iteration t (global counter, from 1):
 * column block s_t = (t-1) mod S, row block r_t drawn uniformly with
 * replacement (SplitMix64 stream 2, draw t-1); on B = I_r x J_s it forms
 * eta = [X,Gamma,U]_I [B,Z,V]_J', mu = g^-1(clamp(eta)), the deviance
 * derivatives D1 = -w(y-mu)/(phi nu g'), D2 = w/(phi nu g'^2) (Section 3),
 * the minibatch gradients of eq. 15 / Appendix B for [Gamma,U]_I and [B,V]_J
 * from the pre-step parameters, the EMAs of eq. 12 (float64) and the step
 * theta -= rho_t alpha_t Gbar / (Hbar + damping) (eq. 13-14).  Unless
 * cfg.skip_block_deviance is set it also records the block deviance
 * sum_B w D(y, mu) (float64, see gmf_block_deviance).  Asynchronous.
 * Errors: GMF_EINVAL (nsteps < 0), GMF_EDEVICE. */
int gmf_step(void* ctx, int64_t nsteps);

/* gmf_compact_counts -- 1 if the step tiles and the full deviance of this
 * context read the 16-bit copy of the counts (cfg.compact_counts, see
 * there), 0 if they read the float32 counts; GMF_EINVAL for a NULL ctx.
 * Host only. */
int gmf_compact_counts(void* ctx);

/* gmf_set_precision -- switch the arithmetic of the following steps and
 * projections (GMF_PREC_FP32 / GMF_PREC_BF16 / GMF_PREC_BF16X3) on the same
 * iterate and moments, e.g. a context fitted in FP32 that projects new rows
 * in BF16X3.  The bfloat16 precisions need a panel stride of 16, 32 or 64
 * (an FP32 context at stride 48 cannot switch).  Errors: GMF_EINVAL (unknown
 * precision, panel stride, tile_waves = 8 not available for it). */
int gmf_set_precision(void* ctx, int32_t precision);

/* gmf_fit -- run epochs of R*S steps (one epoch = R sweeps over J_1..J_S) up
 * to max_epochs; every eval_every epochs evaluate the full deviance and stop
 * when its relative change is below tol (tol <= 0: run all epochs).
 * dev_trace_host (may be NULL) receives one deviance per evaluation (room for
 * max_epochs/eval_every values); *epochs_done_host the epochs run.
 * Returns GMF_OK, GMF_ENOTCONV (tol > 0 not met), GMF_ENUMERIC, GMF_EDEVICE. */
int gmf_fit(void* ctx, int32_t max_epochs, double tol, int32_t eval_every,
            double* dev_trace_host, int32_t* epochs_done_host);

/* gmf_run -- run `epochs` epochs (R*S steps each) and, every eval_every
 * epochs when dev_trace_host is not NULL, the full deviance (as gmf_deviance)
 * of the iterate at that point: on the context's stream between the epochs
 * (cfg.eval_overlap = 0), or on a second stream from a copy of the panels so
 * that it overlaps the following steps (cfg.eval_overlap = 1); the values are
 * the same.  Either way nothing waits for the host.  dev_trace_host
 * receives epochs/eval_every values; eval_ms_host (may be NULL) the time at
 * which each evaluation finished on the device, in ms since the call's work
 * began.  No early stop.  Needs no more workspace than gmf_workspace_bytes
 * gives.  Synchronises at the end (and every 256 evaluations). */
int gmf_run(void* ctx, int32_t epochs, int32_t eval_every, double* dev_trace_host,
            double* eval_ms_host);

/* gmf_deviance -- full deviance sum_ij w_ij D(y_ij, mu_ij) of the current
 * parameters (D as defined after eq. 2, Supplementary Table 1 times 2;
 * NB deviance of Appendix B), accumulated in float64 in a fixed order, and the
 * penalised objective D/(2 phi) + sum_k lambda_k/2 ||theta_k||_F^2 (eq. 6).
 * Either host pointer may be NULL.  Synchronises. */
int gmf_deviance(void* ctx, double* total_host, double* penalized_host);

/* gmf_row_deviance -- the deviance of every row, sum_j w_ij D(y_ij, mu_ij) at
 * the current parameters (the unit deviance D defined after eq. 2,
 * Supplementary Table 1 times 2, NB form of Appendix B: the row terms of the
 * full deviance of gmf_deviance), into per_row (device, n doubles, the
 * caller's row order; caller-owned).  Per entry: eta and the mu part of the
 * unit deviance in float32, the count-only part and the row sums in float64
 * (fixed order); the rows add up to gmf_deviance's total up to the summation
 * order.  Asynchronous on the context's stream.  Errors: GMF_EINVAL (NULL
 * ctx or per_row), GMF_EDEVICE (launch failure). */
int gmf_row_deviance(void* ctx, double* per_row);

/* gmf_block_deviance -- the block deviances of the last `count` steps, oldest
 * first, into host memory (count <= min(steps done, 4096)).  Synchronises.
 * GMF_EINVAL when the context skips them (skip_block_deviance) or when any
 * of the requested steps was run by gmf_batch_run, which forms none. */
int gmf_block_deviance(void* ctx, double* out_host, int64_t count);

/* gmf_get_params -- copy B (m x p), Gamma (n x q), U (n x d), V (m x d) into
 * caller device arrays in original order (any pointer may be NULL to skip).
 * postprocess = 0: the raw iterate.  postprocess = 1: the identifiability
 * projection of Algorithm 2, constraints (A) then (B1), computed in float64
 * on the device (Gram matrices, CholeskyQR2, one-sided Jacobi SVD of the
 * d x d core, sign rule: first non-zero entry of each V column positive);
 * the context's iterate is left unchanged.  Enqueued; synchronises only to
 * check errors. */
int gmf_get_params(void* ctx, float* B, float* A, float* U, float* V,
                   int32_t postprocess);

/* gmf_get_moments -- copy the smoothed gradients/Hessians (float64, original
 * order): Grow, Hrow n x (q+d) for [Gamma, U]; Gcol, Hcol m x (p+d) for
 * [B, V].  Any pointer may be NULL. */
int gmf_get_moments(void* ctx, double* Grow, double* Hrow, double* Gcol,
                    double* Hcol);

/* gmf_set_params -- overwrite the iterate (original order, like gmf_init's
 * starting values); the moments and the step counter are kept. */
int gmf_set_params(void* ctx, const float* B, const float* A, const float* U,
                   const float* V);

/* Saved state (checkpoint and resume of Algorithm 1).  The state of a fit
 * between two steps is: the parameters [Gamma, U] and [B, V] (with the
 * covariates, in the context's permuted panel layout), the four float64
 * smoothed moments of eq. 12, the step counter t (which is also the cursor of
 * the seeded schedule: the partitions and the row-block draws are functions
 * of seed, n, m, R and S) and the ring of the last block deviances.
 * gmf_state_bytes -- host bytes of a saved state of ctx (0 for NULL). */
size_t gmf_state_bytes(void* ctx);
/* gmf_save_state -- write ctx's state into host_buf (caller-owned host
 * memory of at least gmf_state_bytes bytes): a header (format version, shape,
 * family, link, panel stride, schedule seed, step-size and EMA parameters, t)
 * and the device regions, copied after the work queued on ctx's stream.
 * Synchronises.  Errors: GMF_EINVAL (NULL, buffer too small), GMF_EDEVICE. */
int gmf_save_state(void* ctx, void* host_buf, size_t bytes);
/* gmf_load_state -- replace ctx's state by a saved one.  ctx must come from
 * gmf_init with the same Y, X, Z, W and a configuration with the same n, m, d,
 * p, q, R, S, family, link, panel stride, seed, rate0, decay, tau, alpha1,
 * alpha2 and damping (the starting values passed to gmf_init do not matter);
 * else GMF_EINVAL and ctx is unchanged.  Steps run after the load continue
 * the saved run exactly: the same blocks, step sizes and results, bit for bit,
 * as if it had not been interrupted.  Synchronises. */
int gmf_load_state(void* ctx, const void* host_buf, size_t bytes);

/* gmf_initialize_workspace_bytes -- device bytes gmf_initialize needs for a
 * test matrix of k columns (0 for NULL ctx or k outside [d, 64]). */
size_t gmf_initialize_workspace_bytes(void* ctx, int32_t k);
/* gmf_initialize -- the paper's parameter initialization (Section 4.1,
 * "Parameter initialization"), in the least-squares form the paper gives for
 * high-dimensional data, computed on the device into the context's iterate:
 *   1. B' = (X'X)^-1 X'L with L = g(y + c) (the m column regressions);
 *   2. Gamma = (L - X B') Z (Z'Z)^-1 (the n row regressions given the column
 *      offsets);
 *   3. U: the d leading left singular vectors of the residual matrix E at
 *      mu~ = g^-1(X B' + Gamma Z') (clamped like the fit's mean), Pearson
 *      residuals (y - mu~) sqrt(w / nu(mu~)) (residual = 0) or deviance
 *      residuals sign(y - mu~) sqrt(w D(y, mu~)) (residual = 1), by a
 *      randomized range finder (Halko, Martinsson and Tropp 2011): Y = E Omega,
 *      power_iters times Y = E orth(E' orth(Y)), Q = orth(Y), then the left
 *      singular vectors of Q'E mapped back by Q;
 *   4. V' = (U'U)^-1 U' (L - X B' - Gamma Z') (the column regressions of the
 *      link-scale residual on the scores);
 *   then each pair (u_k, v_k) is rescaled to equal norms (U V' unchanged).
 * No n x m matrix is stored: every pass forms its entries from Y on the fly;
 * sums are float32 within 64-entry tiles and float64 across tiles (fixed
 * order); orthonormalisation (two rounds of Cholesky QR), the normal
 * equations and the small eigenproblem are float64.
 *   ws / ws_bytes: caller device workspace (gmf_initialize_workspace_bytes).
 *   Omega: m x k float32 test matrix (device, the caller's column order;
 *     normally standard Gaussian draws), d <= k <= 64.
 *   y_offset: c in g(y + c); < 0 selects 1/2 for the log link, 0 for the
 *     identity link; the log link needs c > 0.
 * Needs p + q <= 32 and no step run yet (t = 0); the moments stay zero.
 * Synchronises.  Errors: GMF_EINVAL, GMF_EWORKSPACE, GMF_ENUMERIC (X'X,
 * Z'Z or U'U not positive definite, or the range finder's basis lost rank),
 * GMF_EDEVICE. */
int gmf_initialize(void* ctx, void* ws, size_t ws_bytes, const float* Omega, int32_t k,
                   int32_t power_iters, int32_t residual, double y_offset);

/* gmf_set_column_alpha -- give the NB family one shape per column: alpha
 * (device, m positive floats, the caller's column order) replaces the scalar
 * cfg.nb_alpha in D1, D2 and the deviance of every following step and
 * evaluation (Appendix B's NB law, with alpha_j per column).  The context then
 * runs the generic FP32 epilogue.  Errors: GMF_EINVAL (not NB, NB shape being
 * estimated, precision not FP32, a value not positive and finite). */
int gmf_set_column_alpha(void* ctx, const float* alpha);

/* gmf_get_dispersion -- the dispersion phi and NB shape in use: the
 * configured values, or the current estimates when cfg.estimate_phi /
 * cfg.estimate_alpha are set.  Either pointer may be NULL.  Synchronises. */
int gmf_get_dispersion(void* ctx, double* phi_host, double* alpha_host);

/* gmf_heldout_metrics -- the out-of-sample reconstruction errors of Section
 * 5.2 for entries held out of the fit.  Ytest (device, n x m, the caller's
 * order, y_dtype as in gmf_init) holds the held-out values; every other entry
 * is marked by a negative int32 or a NaN float32.  With ybar_T the mean of
 * the observed entries of the context's Y and mu the fitted means:
 *   out_host[0] = sum [log((1+y)/(1+mu))]^2 / sum [log((1+y)/(1+ybar_T))]^2,
 *   out_host[1] = sum D_Poisson(y, mu) / sum D_Poisson(y, ybar_T),
 *   out_host[2] the same ratio with the context family's deviance,
 *   out_host[3] the number of held-out entries, out_host[4] ybar_T,
 *   out_host[5] the number of observed training entries.
 * Sums over the held-out entries; per entry float32, float64 sums in a fixed
 * order.  Synchronises.  Errors: GMF_EINVAL, GMF_EDEVICE. */
int gmf_heldout_metrics(void* ctx, const void* Ytest, int32_t y_dtype, double* out_host);

/* Rank selection (Section 4.2, "Model selection").
 * gmf_init_spectrum -- the `count` largest singular values (descending) of
 * the residual matrix that the last gmf_initialize on ctx factored (the
 * Pearson or deviance residuals after the least-squares column and row
 * effects; the paper's scree plot uses their squares), as estimated by its
 * range finder; count <= that call's k.  GMF_EINVAL before any
 * initialization. */
int gmf_init_spectrum(void* ctx, double* sv_host, int32_t count);
/* gmf_rank_eigengap -- the eigenvalue-gap ("edge distribution") estimator of
 * Onatski (2010, Review of Economics and Statistics 92(4)) on host
 * eigenvalues lambda_1 >= ... >= lambda_count (count >= rmax + 5): from
 * j = rmax + 1, delta = 2 |slope| of the least-squares line of
 * lambda_j..lambda_{j+4} on (j-1)^{2/3}..(j+3)^{2/3}; rank = the largest
 * i <= rmax with lambda_i - lambda_{i+1} >= delta (0 if none); j = rank + 1;
 * repeated until the rank no longer changes.  Pure host computation.
 * Errors: GMF_EINVAL (NULL, count too small, not sorted or not finite). */
int gmf_rank_eigengap(const double* eigenvalues, int32_t count, int32_t rmax, int32_t* rank_host);
/* gmf_rank_select_cv -- the out-of-sample criterion: dev_host[r * nfolds + f]
 * is the held-out deviance (gmf_heldout_metrics) of candidate r's fit on fold
 * f; *best_host = the candidate with the smallest mean over the folds (the
 * first on ties).  Pure host computation. */
int gmf_rank_select_cv(const double* dev_host, int32_t nranks, int32_t nfolds, int32_t* best_host);

/* gmf_get_schedule -- the drawn schedule, for checking: row_perm_host (n) and
 * col_perm_host (m) receive the permutations (block r holds
 * row_perm[floor(rn/R) .. floor((r+1)n/R)-1]); r_host receives the row
 * blocks of steps t_first .. t_first+count-1 (t from 1).  Any may be NULL. */
int gmf_get_schedule(void* ctx, int32_t* row_perm_host, int32_t* col_perm_host,
                     int64_t t_first, int64_t count, int32_t* r_host);

/* gmf_schedule_host -- the same schedule without a context or device (host
 * arrays): the permutations of gmf_init for (seed, n, m) and the row blocks
 * r_t of steps t_first .. t_first+count-1 for R row blocks.  Any output may
 * be NULL.  Pure host computation. */
int gmf_schedule_host(uint64_t seed, int64_t n, int64_t m, int32_t R, int64_t t_first,
                      int64_t count, int32_t* row_perm_host, int32_t* col_perm_host,
                      int32_t* r_host);

/* gmf_set_timing -- enable (1) or disable (0) HIP-event timing of the step
 * launches on the context's stream: each subsequent launch of the step kernel
 * (one per gmf_step call, or per 8192 steps) is bracketed by events.
 * gmf_get_timing synchronises and returns, for the launches since the last
 * call, the summed launch time in milliseconds, the number of launches and
 * the number of steps they ran, then starts a new window.  Any output may be
 * NULL. */
int gmf_set_timing(void* ctx, int32_t enable);
int gmf_get_timing(void* ctx, double* launch_ms_host, double* launches_host,
                   int64_t* steps_host);

/* gmf_get_timing_by_kind -- the same window split by launch kind, without
 * starting a new one: ms_host[0], launches_host[0] for the launches that run
 * block-step tiles (the tiles of a level, with any updates that share the
 * launch: the step kernel), [1] for the update-only launches (the update
 * kernel).  Both arrays hold 2 doubles.  Synchronises.  Errors: GMF_EINVAL
 * (NULL argument). */
int gmf_get_timing_by_kind(void* ctx, double* ms_host, double* launches_host);

/* gmf_project_workspace_bytes -- device bytes gmf_project needs for n_new
 * new rows of the context's shape (0 on error). */
size_t gmf_project_workspace_bytes(void* ctx, int64_t n_new);

/* gmf_project -- fit the row side [Gamma, U] of n_new new rows with the column
 * side frozen (B, Z, V of the context), by the row half of Algorithm 1 (its
 * step 4, with the covariate form of Appendix B): step t (from 1) uses every
 * new row and column block J_{(t-1) mod S} of the context's partition,
 * G = (m/|J|) D1 [Z,V]_J + lambda [0_A, U] style ridge terms as in gmf_step,
 * float64 EMAs starting at zero, step rho_t alpha_t Gbar/(Hbar + damping).
 * Rows are independent (the objective is convex in each row given V, eq. 7).
 *   ws / ws_bytes: caller device workspace (gmf_project_workspace_bytes).
 *   Ynew n_new x m (y_dtype as in gmf_init), Xnew n_new x p (NULL if p = 0).
 *   A0 n_new x q, U0 n_new x d: starting values.
 *   epochs: S steps each.  frozen = 0: the context's raw iterate; 1: its
 *   Algorithm 2 (A + B1) projection, computed in float64.
 *   A_out, U_out (device, may alias A0/U0): results.  dev_trace_host (may be
 *   NULL): epochs + 1 values, the deviance of the new rows before the first
 *   step and after every epoch.
 * The steps run in the context's current precision (gmf_set_precision), one
 * launch per step: each wavefront steps its own rows over the whole column
 * block, so the gradient sums accumulate in float32 over the block in matrix-
 * core order (the fit sums per 128-column strip, then over strips in float64).
 * Enqueued on the context's stream; synchronises when dev_trace_host is set.
 * The context's own iterate is not changed. */
int gmf_project(void* ctx, void* ws, size_t ws_bytes, const void* Ynew, int32_t y_dtype,
                int64_t n_new, const float* Xnew, const float* A0, const float* U0,
                int32_t epochs, int32_t frozen, float* A_out, float* U_out,
                double* dev_trace_host);

/* gmf_project_warm -- gmf_project with its starting values built on the
 * device, for a learned warm start of new rows (scores predicted from the
 * counts, e.g. by the encoder below):
 *   Gamma_0: the first column (Z's first column must be the intercept, z_j0 =
 *     1) matches the row total given the frozen X B' part: log link
 *     gamma_i0 = log(sum_j y_ij + 1/2) - log sum_j exp(x_i' beta_j); identity
 *     link gamma_i0 = mean_j (y_ij - x_i' beta_j); other columns 0.
 *   U_0: per row, U_cand's row when its row deviance sum_j D(y_ij, mu_ij)
 *     (with Gamma_0) is below that of u_i = 0, else 0 (a fallback row).
 *     U_cand NULL: U_0 = 0 for every row (the cold start).
 * Then `epochs` epochs as in gmf_project.  Arguments as in gmf_project, and
 *   U_cand (device, n_new x d, or NULL);
 *   epoch_ms_host (may be NULL; needs dev_trace_host): epochs + 1 values, the
 *     wall milliseconds since the call began at each deviance evaluation;
 *   fallback_rows_host (may be NULL): the number of fallback rows.
 * Same workspace as gmf_project.  With epochs = 0, A_out / U_out receive the
 * starting values. */
int gmf_project_warm(void* ctx, void* ws, size_t ws_bytes, const void* Ynew, int32_t y_dtype,
                     int64_t n_new, const float* Xnew, const float* U_cand, int32_t epochs,
                     int32_t frozen, float* A_out, float* U_out, double* dev_trace_host,
                     double* epoch_ms_host, int64_t* fallback_rows_host);

/* gmf_project_noalloc -- gmf_project without a workspace argument and without
 * any device allocation, for callers that cannot allocate (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc).  The
 * projection's scratch (the new rows' block layout, panels, moments, deviance
 * partials) lives in a resident 64 MiB device array of the library, one per
 * device, held until the process ends; its address is taken at gmf_init.
 * Limit: gmf_project_workspace_bytes(ctx, n_new) must be <= 64 MiB (about
 * 8,000 new rows of 2,000 columns, about 5,000 when the context keeps the
 * 16-bit counts), else GMF_EWORKSPACE.  Every call on a
 * device shares that device's array and overwrites it: calls that overlap on
 * one device (several streams or threads) race and must be serialised by the
 * caller.  Arguments, results and the other errors as gmf_project. */
int gmf_project_noalloc(void* ctx, const void* Ynew, int32_t y_dtype, int64_t n_new,
                        const float* Xnew, const float* A0, const float* U0, int32_t epochs,
                        int32_t frozen, float* A_out, float* U_out, double* dev_trace_host);

/* ---------------------------------------------------------------------------
 * Batched fits.  Many independent contexts (each from gmf_init, any shapes,
 * Poisson / NB / Gaussian mixed) advance together: one epoch of the batch is
 * a fixed sequence of launches -- for k = 0, 1, ..., the tiles of step k of
 * every fit, then the updates of step k -- so each fit's steps run in order
 * exactly as gmf_step runs them (same results, the block deviance of each
 * step is not formed), while the fits share every launch.  The random row
 * blocks and step sizes of the coming epochs are uploaded as a device table,
 * so the launch sequence of an epoch is the same every epoch; with use_graph
 * it is recorded once as a HIP graph and replayed.  All contexts must share
 * the precision and the panel stride (gmf_config.panel_stride) and live on one
 * device; they must stay alive, and must not be used on their own while a
 * gmf_batch_run call is in progress.  The batch runs on a stream of its own,
 * ordered after the work already queued on the contexts' streams, and their
 * streams are ordered after it.
 * ------------------------------------------------------------------------- */
/* Device bytes of the batch workspace (0 on invalid arguments). */
size_t gmf_batch_workspace_bytes(void* const* ctxs, int32_t nfits, int32_t table_epochs);
/* gmf_batch_init -- set up a batch over ctxs[0..nfits) with a step table of
 * table_epochs epochs (refilled from the host when used up: one stream
 * synchronisation per refill).  mode 0: the fixed launch sequence above,
 * launched directly; 1: the same sequence recorded once as a HIP graph and
 * replayed; 2: level placement -- each fit's steps of a table are placed by
 * the rule of a single fit (gmf_step: a step waits only for the previous steps
 * on its row block, column block and partial slot), so launch k runs the
 * tiles of every fit's level-k steps and the updates of every fit's
 * level-(k-1) steps (about 27 launches per epoch of R = 10, S = 5 fits
 * instead of 100), launched directly.  All modes give the results of stepping
 * each fit on its own.  Errors: GMF_EINVAL (mixed precision / panel stride,
 * repeated or NULL contexts, a fit that estimates its dispersion, bad mode),
 * GMF_EWORKSPACE, GMF_EDEVICE. */
int gmf_batch_init(void** batch_out, void* const* ctxs, int32_t nfits, void* ws,
                   size_t ws_bytes, int32_t table_epochs, int32_t mode);
/* gmf_batch_run -- run `epochs` epochs of every fit (fit f: R_f * S_f steps
 * each).  Every eval_every epochs, when dev_trace_host is not NULL, the full
 * deviance of every fit is evaluated (float64, as gmf_deviance) into
 * dev_trace_host[f * (epochs / eval_every) + i]; this synchronises.  Errors as
 * gmf_step, GMF_ENUMERIC when a fit produced a non-finite parameter. */
int gmf_batch_run(void* batch, int32_t epochs, int32_t eval_every, double* dev_trace_host);
void gmf_batch_destroy(void* batch);

/* ---------------------------------------------------------------------------
 * Tile autotuning.  The rows per step tile (gmf_config.tile_rows) trade the
 * parallelism of a step against the partial sums its tiles write; the best
 * value depends on the block shape.  gmf_tune measures candidates and records
 * the fastest in a process-wide table keyed by (precision, family, panel
 * stride, ceil(log2 |I|), ceil(log2 |J|)) with |I| = ceil(n/R), |J| = ceil(m/S);
 * gmf_workspace_bytes and gmf_init use the table when tile_rows = 0 (else the
 * automatic rule).  The table can be saved to and loaded from a text file.
 * ------------------------------------------------------------------------- */
/* gmf_tune -- for each candidate tile_rows (multiples of 32): gmf_init a
 * context with it in ws (ws_bytes must cover gmf_workspace_bytes for every
 * candidate), run min(steps, R*S) warm-up steps, time `steps` steps with HIP
 * events on `stream`, destroy it.  us_per_step_host (may be NULL) receives
 * ncand times; *best_host the fastest candidate, which is stored in the table.
 * Inputs as in gmf_init.  Synchronises. */
int gmf_tune(const gmf_config* cfg, void* ws, size_t ws_bytes, void* stream, const void* Y,
             int32_t y_dtype, const float* X, const float* Z, const float* W, const float* B0,
             const float* A0, const float* U0, const float* V0, const int32_t* candidates,
             int32_t ncand, int32_t steps, int32_t* best_host, double* us_per_step_host);
/* The table's tile_rows for cfg's class, or 0 when it has none. */
int32_t gmf_tune_lookup(const gmf_config* cfg);
void gmf_tune_table_clear(void);
/* Text file, one class per line: precision family panel_stride log2|I| log2|J|
 * tile_rows us_per_step; '#' starts a comment line.  Load merges into the
 * table (GMF_EINVAL on a malformed line, the table unchanged). */
int gmf_tune_table_save(const char* path);
int gmf_tune_table_load(const char* path);

/* ---------------------------------------------------------------------------
 * Warm-start encoder.  An MLP maps a row's counts to its latent scores:
 * x = log(1 + y_i) (m values) -> Linear(m, H) -> GELU -> Linear(H, H) -> GELU
 * -> Linear(H, d), GELU(z) = z Phi(z).  It is trained on (row, fitted u_i)
 * pairs by minimising the mean squared error with Adam (bias-corrected
 * moments, optional decoupled weight decay) in float32 on the matrix cores,
 * and runs inference with bfloat16 operands (float32 accumulation) or float32.
 * The weights live in the caller's workspace; the layout of each weight is
 * row-major (out x in); biases are vectors.
 * ------------------------------------------------------------------------- */
typedef struct gmf_mlp_config {
  int32_t m;          /* input width (columns of Y)                      */
  int32_t hidden;     /* hidden width H                                   */
  int32_t d;          /* output width (rank)                              */
  int32_t batch;      /* minibatch rows per Adam step                     */
  double lr, beta1, beta2, eps, weight_decay;
} gmf_mlp_config;

/* Defaults: m=1, hidden=256, d=1, batch=256, lr=1e-3, beta1=0.9,
 * beta2=0.999, eps=1e-8, weight_decay=0. */
void gmf_mlp_config_default(gmf_mlp_config* cfg);
/* Device workspace bytes of an encoder (0 for an invalid cfg). */
size_t gmf_encoder_workspace_bytes(const gmf_mlp_config* cfg);
/* gmf_encoder_init -- copy the starting weights (device arrays: W1 H x m,
 * b1 H, W2 H x H, b2 H, W3 d x H, b3 d) into the workspace and zero the Adam
 * moments.  Synchronises.  Errors: GMF_EINVAL, GMF_EWORKSPACE, GMF_EDEVICE. */
int gmf_encoder_init(void** enc_out, const gmf_mlp_config* cfg, void* ws, size_t ws_bytes,
                     void* stream, const float* W1, const float* b1, const float* W2,
                     const float* b2, const float* W3, const float* b3);
/* gmf_encoder_train -- `epochs` passes over nrows (Y row-major nrows x m,
 * y_dtype as in gmf_init; U nrows x d targets), minibatches of cfg.batch
 * consecutive rows in the given order, one Adam step per minibatch.
 * loss_trace_host (may be NULL): the mean training loss of every epoch
 * (synchronises once per epoch when given). */
int gmf_encoder_train(void* enc, const void* Y, int32_t y_dtype, const float* U, int64_t nrows,
                      int32_t epochs, double* loss_trace_host);
/* gmf_encoder_forward -- U_out (nrows x d, device) = encoder(Y).  bf16 = 0:
 * float32 operands; 1: bfloat16 operands, all three layers fused in one
 * kernel (64 rows per workgroup, activations kept on chip) when hidden is a
 * multiple of 64 up to 256 and d <= 64, else layer by layer; 2: bfloat16
 * operands layer by layer (same products and rounding as 1).  Enqueued. */
int gmf_encoder_forward(void* enc, const void* Y, int32_t y_dtype, int64_t nrows, float* U_out,
                        int32_t bf16);
/* gmf_encoder_loss_grad -- for one minibatch (nrows <= cfg.batch) compute the
 * mean squared error and its gradient without updating: grad_out (device, may
 * be NULL) receives the flat gradient [W1, b1, W2, b2, W3, b3] in the weight
 * layouts above.  Synchronises. */
int gmf_encoder_loss_grad(void* enc, const void* Y, int32_t y_dtype, const float* U, int64_t nrows,
                          double* loss_host, float* grad_out);
/* Copy the current weights out (device arrays, any may be NULL). */
int gmf_encoder_get_weights(void* enc, float* W1, float* b1, float* W2, float* b2, float* W3,
                            float* b3);
void gmf_encoder_destroy(void* enc);
/* Message for the last failing encoder call on this thread. */
const char* gmf_encoder_last_error(void);

/* gmf_set_trace -- record a timeline of the step launches into a caller
 * device buffer of `records` x 8 uint64 (NULL disables).  Every workgroup of
 * the following level launches that has work writes one record at index
 * (workgroups of earlier traced launches) + its workgroup index:
 * [0] launch number, [1] (workgroup << 32) | kind (0 tile, 1 row update,
 * 2 column update, 3 block-deviance sum), [2] start and [3] end stamp
 * (s_memrealtime, 100 MHz), [4] hardware compute-unit id, [5..7] for tiles
 * the stamps after its operand loads, after its first row group's U side and
 * after its last row group (else 0).  Workgroups without work leave their
 * record untouched; records past the capacity are dropped.  For profiling
 * only. */
int gmf_set_trace(void* ctx, void* buffer, int64_t records);

/* Steps run so far (the global counter t of the last step). */
int64_t gmf_steps_done(void* ctx);

/* gmf_sync -- wait for the context's stream and report GMF_ENUMERIC if a
 * non-finite value was produced since the last check (the flag is cleared). */
int gmf_sync(void* ctx);

/* Release the context (not the workspace). NULL is ignored. */
void gmf_destroy(void* ctx);

/* Message for the last failing call on this thread ("" if none). */
const char* gmf_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* GMF_H_ */
