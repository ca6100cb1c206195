/*
 * hsim.h -- C ABI of the hierarchical-simulation CVA library (libhsim.so, gfx950).
 *
 * The library computes the data-parallel path of the hierarchical ("oversimulated")
 * CVA scheme of Abbas-Turki, Crepey & Saadeddine, "Pathwise CVA regressions with
 * oversimulated defaults":
 *   - M outer paths of the market factors (Vasicek short rates, log-normal FX rates,
 *     CIR default intensities; Appendix B, equations e:sde1 and e:sde2) are stepped
 *     by Euler on a fine grid (Section 4.1, remark rem:finecoarse);
 *   - every swap is priced at every pricing date with the three-case formula of
 *     Appendix B, and the exposures D^c_j = LGD_c beta_j (MtM^c_j)^+ are formed;
 *   - each outer path carries n_b inner default draws (Section 3.2), with the default
 *     rule of equation e:tau checked at pricing dates;
 *   - the pathwise CVA loss of eq:CVA_portfolio is averaged over the inner draws
 *     into the regression targets T_i, and CVA_0 = mean_k T^k_0;
 *   - the targets are regressed onto the market state by NN^+ networks (e:nnp),
 *     trained by BaseAlg (Algorithm 1) and Backward learning (Algorithm 2);
 *   - the sensitivities of CVA_0 to the model parameters are computed by an adjoint
 *     sweep of the smoothed (conditional) estimator.
 *
 * Conventions
 *   - Every entry point returns an int status: HSIM_OK (0) or a negative error code.
 *     A message for the last error of the calling thread is in hsim_last_error().
 *     No C++ exception crosses the ABI.
 *   - Pointers named *_dev are device memory owned by the caller (for instance torch
 *     tensors); the library never frees or keeps them.  Host structs and host arrays
 *     are read only during the call.
 *   - Work is enqueued on `stream` (a hipStream_t passed as void*, NULL = default
 *     stream) and is asynchronous unless stated otherwise.
 *   - Results depend only on the inputs, the seed and global path/draw indices: never
 *     on grid or block sizes, nor on how a path range is split over calls.
 *   - Arrays are dense and row-major in the index order written, e.g. [n+1][C][M]
 *     means element (j, c, k) at offset (j*C + c)*M + k.
 *   - Arguments are validated before any launch: a null pointer, a non-positive size,
 *     a correlation matrix that is not positive definite, a reset period that is not a
 *     whole number of pricing steps, sizes beyond the stated limits, or a workspace
 *     that is too small return an error and launch nothing.
 */
#ifndef HSIM_H
#define HSIM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define HSIM_ABI_VERSION 3

enum hsim_status {
  HSIM_OK = 0,
  HSIM_EINVAL = -1,       /* bad argument */
  HSIM_ERANGE = -2,       /* a size beyond the supported limits */
  HSIM_ENOWS = -3,        /* workspace too small */
  HSIM_EDEVICE = -4,      /* a HIP runtime call failed */
  HSIM_EUNSUPPORTED = -5, /* a shape the library was not built for */
  HSIM_ETIMEOUT = -6      /* a bounded device-side wait gave up; the results are incomplete */
};

/* Arithmetic of the simulation.  HSIM_FP64: all state and prices in FP64.  HSIM_FP32:
 * state, normals and prices in FP32; the integrals int r^0 and int gamma^c (hence
 * beta and Lambda) are accumulated in FP64.  HSIM_FP32_PLAIN (hsim_outer_paths and
 * hsim_inner_defaults_cva only; the baseline the FP64-integral form is measured against): as
 * HSIM_FP32 but the integrals, beta and the exposures' discounting are FP32 too; its outputs have
 * the FP32 types (I and Lambda are still written as double). */
enum hsim_precision { HSIM_FP64 = 0, HSIM_FP32 = 1, HSIM_FP32_PLAIN = 2 };

/* Regression inputs emitted per date.  FACTORS: r^0..r^{n_e-1}, log chi^1..log chi^{n_e-1},
 * gamma^1..gamma^C (the diffusive factors of Section 4.3).  FACTORS_PLUS adds
 * I_i = -log beta_i and sum_c Lambda^c_i. */
enum hsim_features { HSIM_FEAT_FACTORS = 0, HSIM_FEAT_FACTORS_PLUS = 1 };

/* Limits of this build. */
#define HSIM_MAX_CCY 16
#define HSIM_MAX_CPTY 16
#define HSIM_MAX_BRANCH (1 << 24)
#define HSIM_MAX_DATES 512
#define HSIM_MAX_PERIODS 64

/* Model parameters (Appendix B).  Host pointers.  Brownian ordering of `corr`
 * (dimension d_W = 2 n_ccy - 1, row-major, symmetric positive definite, unit
 * diagonal): index e < n_ccy drives r^e, index n_ccy + e - 1 drives log chi^e for
 * 1 <= e < n_ccy.  The correlation rho^e of (r^e, log chi^e) enters the drift of r^e
 * under the domestic measure as -rho^e sigma_r^e sigma_fx^e.  CIR drivers are
 * independent of the market block and of each other. */
typedef struct {
  int32_t n_ccy;              /* 1 <= n_ccy <= HSIM_MAX_CCY; currency 0 is the reference */
  int32_t n_cpty;             /* 1 <= n_cpty <= HSIM_MAX_CPTY */
  const double* a;            /* [n_ccy] Vasicek speed (> 0) */
  const double* b;            /* [n_ccy] Vasicek level under Q^e */
  const double* sigma_r;      /* [n_ccy] Vasicek volatility (>= 0) */
  const double* r0;           /* [n_ccy] initial short rates */
  const double* sigma_fx;     /* [n_ccy-1] FX log-volatility (>= 0); may be NULL if n_ccy = 1 */
  const double* fx0;          /* [n_ccy-1] initial FX rates (> 0); may be NULL if n_ccy = 1 */
  const double* corr;         /* [(2 n_ccy - 1)^2] */
  const double* kappa;        /* [n_cpty] CIR speed */
  const double* theta;        /* [n_cpty] CIR level */
  const double* nu;           /* [n_cpty] CIR volatility (>= 0) */
  const double* lambda0;      /* [n_cpty] initial intensity (>= 0) */
  const double* lgd;          /* [n_cpty] loss given default */
} hsim_market;

/* Swap book (Appendix B): spot-starting swaps, resets every `delta` years, paying fixed
 * delta*fixed_rate and receiving floating 1/ZC_{t-}(t) - 1 at every reset date but 0.
 * payer = +1: the bank pays fixed; payer = -1: the bank receives fixed.  Notionals are
 * in the swap's currency.  Host pointers. */
typedef struct {
  int32_t n_swaps;            /* >= 1 */
  const int32_t* ccy;         /* [n_swaps] in [0, n_ccy) */
  const int32_t* cpty;        /* [n_swaps] in [0, n_cpty) */
  const int32_t* periods;     /* [n_swaps] maturity in reset periods, 1..HSIM_MAX_PERIODS */
  const double* notional;     /* [n_swaps] */
  const double* fixed_rate;   /* [n_swaps] swap rate Sigma */
  const int32_t* payer;       /* [n_swaps] +1 or -1 */
  double delta;               /* reset period in years (> 0) */
} hsim_portfolio;

/* Time grid: n_dates pricing dates t_i = i*horizon/n_dates, n_sub Euler sub-steps each.
 * delta*n_dates/horizon must be a whole number q (pricing steps per reset period), and
 * every maturity must lie within the horizon. */
typedef struct {
  double horizon;
  int32_t n_dates;            /* 1..HSIM_MAX_DATES */
  int32_t n_sub;              /* >= 1 */
} hsim_grid;

int hsim_abi_version(void);
const char* hsim_last_error(void);

/* Number of regression inputs per date for a feature mode. */
int hsim_n_features(const hsim_market* market, int feature_mode);

/* Time-0 par rates of the swaps (the fixed rate that makes the t = 0 case of the
 * Appendix B swap price vanish), in host memory: par_out[n_swaps].  Synchronous. */
int hsim_par_rates(const hsim_market* market, const hsim_portfolio* book, double* par_out);

/* Test hook: the raw Philox4x32-10 words of counters (k, c1, c2, c3) for
 * k = k_begin .. k_begin+count-1, with key (seed mod 2^32, seed >> 32):
 * out_dev[4*(k-k_begin) + w] = word w.  out_dev holds 4*count uint32. */
int hsim_philox_fill(uint64_t seed, uint32_t c1, uint32_t c2, uint32_t c3, int64_t k_begin,
                     int64_t count, uint32_t* out_dev, void* stream);

/* Test hook: the standard normals that outer path k uses at global sub-step s,
 * out_dev[(k - path_begin)*n_z + f] for f < n_z, in the given precision (float or
 * double elements). */
int hsim_normals_fill(uint64_t seed, int64_t path_begin, int64_t count, int32_t s, int32_t n_z,
                      int precision, void* out_dev, void* stream);

/* Outer simulation and pricing (Appendix B; Section 4.1 rem:finecoarse; Section 4.2).
 * Simulates outer paths k = path_begin .. path_begin+M-1 and writes, at every pricing
 * date j = 0..n (n = grid->n_dates):
 *   features_dev [n+1][d][M]   regression inputs (float if FP32, double if FP64); may be NULL
 *   I_dev        [n+1][M]      int_0^{t_j} r^0 (double), beta_j = exp(-I_j); must not be NULL
 *   Lambda_dev   [n+1][C][M]   int_0^{t_j} gamma^{c,+} (double); must not be NULL
 *   D_dev        [n+1][C][M]   LGD_c beta_j (MtM^c_j)^+ (float if FP32, double if FP64); must not be NULL
 *   MtM_dev      [n+1][C][M]   MtM^c_j in the reference currency (same type); may be NULL
 * No workspace is needed. */
int hsim_outer_paths(const hsim_market* market, const hsim_portfolio* book, const hsim_grid* grid,
                     uint64_t seed, int64_t path_begin, int64_t M, int precision, int feature_mode,
                     void* features_dev, double* I_dev, double* Lambda_dev, void* D_dev,
                     void* MtM_dev, void* stream);

/* Inner default draws (Section 3.2; Appendix B e:tau).  For every outer path k of the
 * range and counterparty c, draws l = 0..n_b(k)-1 use the Philox word (k, l>>2, c, 1)
 * [l&3] -> u = (2 floor(word/2^9) + 1) 2^-24, and default at
 *   j* = min{ j >= 1 : Lambda^c_j >= -log u }   (no default if none).
 * counts_dev [n+1][C][M] (int32) receives the number of draws defaulting at each date.
 * n_b(k) = n_b when n_b_per_block is NULL; otherwise path k uses
 * n_b_per_block[(k - path_begin) / block_paths] (device array of ceil(M/block_paths)
 * entries, block_paths a positive multiple of 64).  1 <= n_b(k) <= 2^24.  Uneven n_b runs as
 * one persistent launch that takes the 64-path tiles longest-first (tiles bucketed by
 * floor(log2 n_b)); it needs hsim_workspace_bytes(HSIM_OP_INNER, ...) bytes of device
 * workspace (HSIM_ENOWS otherwise).  Uniform n_b needs none (workspace may be NULL).  The
 * counts do not depend on the schedule. */
int hsim_inner_defaults(const hsim_grid* grid, int32_t n_cpty, uint64_t seed, int64_t path_begin,
                        int64_t M, int32_t n_b, const int32_t* n_b_per_block, int32_t block_paths,
                        const double* Lambda_dev, int32_t* counts_dev, void* workspace_dev,
                        size_t ws_bytes, void* stream);

/* Targets and CVA_0 (Section 4.2 eq:CVA_portfolio; Section 3.2): with the default counts
 * of hsim_inner_defaults,
 *   T_i = exp(I_i) / n_b(k) * sum_{j=i+1}^{n} sum_c D^c_j counts^c_j,   T_n = 0,
 * which is the inner average of the pathwise loss xi_i.  target_dev [n+1][M] (float if
 * FP32, double if FP64).  cva0_dev (one double, device) receives mean_k T^k_0 over the
 * range, reduced in a fixed order.  n_b / n_b_per_block / block_paths as above.
 * Needs hsim_workspace_bytes(HSIM_OP_TARGETS, ...) bytes of device workspace. */
int hsim_targets_cva(const hsim_grid* grid, int32_t n_cpty, int64_t M, int32_t n_b,
                     const int32_t* n_b_per_block, int32_t block_paths, int precision,
                     const double* I_dev, const void* D_dev, const int32_t* counts_dev,
                     void* target_dev, double* cva0_dev, void* workspace_dev, size_t ws_bytes,
                     void* stream);

/* hsim_targets_cva for callers that cannot allocate device memory (code under HIP graph capture,
 * serving loops, harnesses that forbid hipMalloc): the same computation and results, with the
 * FP64 block partials of CVA_0 kept in a static device array that the library holds on every GPU
 * it runs on until the process ends (512 KiB), so no workspace is passed and nothing is
 * allocated.  M <= 2^24 paths (HSIM_ERANGE beyond).  All calls on one GPU share that array: calls
 * that overlap on one GPU (concurrent streams, threads) race and must be ordered by the caller.
 * Other arguments as hsim_targets_cva. */
int hsim_targets_cva_noalloc(const hsim_grid* grid, int32_t n_cpty, int64_t M, int32_t n_b,
                             const int32_t* n_b_per_block, int32_t block_paths, int precision,
                             const double* I_dev, const void* D_dev, const int32_t* counts_dev,
                             void* target_dev, double* cva0_dev, void* stream);

/* The paper's per-inner-sample regression data (Section 3.2: Algorithm 2 on the hierarchical
 * sample I = {paths} x {draws}, inputs (X_i, Y_i) with X the default indicators).  For every
 * outer path k of [path_begin, path_begin + M) and inner draw l < n_b (the draws of
 * hsim_inner_defaults: same Philox words, same default rule), sample r = l M + (k - path_begin)
 * (the order whose contiguous slices are the paper's minibatches) gets at every date i
 *   X_dev[i][f][r] = features_dev[i][f][k]             f < d  (market state Y^k_i)
 *   X_dev[i][d + c][r] = 1{j*_c <= i}                  c < C  (default indicators X^{k,l}_i)
 *   Y_dev[i][r] = exp(I_i) sum_{c : j*_c > i} D^c_{j*_c}     (the pathwise loss xi^{k,l}_i)
 * X_dev [n+1][d + C][n_b M] and Y_dev [n+1][n_b M] are float; features_dev [n+1][d][M] and D_dev
 * as hsim_outer_paths of the same precision (d = 0: indicators only).  M * n_b <= 2^31.  The
 * rows feed cva_regress_fit with M' = n_b M rows and n_feat = d + C (the network takes at most
 * 32 inputs).  No workspace. */
int hsim_sample_rows(const hsim_grid* grid, int32_t n_cpty, int32_t d, uint64_t seed,
                     int64_t path_begin, int64_t M, int32_t n_b, int precision,
                     const void* features_dev, const double* I_dev, const double* Lambda_dev,
                     const void* D_dev, float* X_dev, float* Y_dev, void* stream);

/* Grouped per-inner-sample targets for one counterparty (Section 3.2 with X the default
 * indicator; Algorithm 1's loss over all (path, draw) samples).  A draw whose client has
 * defaulted by t_i has nothing left to lose, and over the A_i draws still alive at t_i the sum
 * of squares equals A_i (phi - mean)^2 plus a constant, so the paper's regression on the alive
 * branch is the weighted regression of
 *   target_dev[i][k] = exp(I_i) / A_i * sum_{j=i+1}^{n} D_j counts_j     (0 when A_i = 0),
 *   weight_dev[i][k] = A_i / n_b(k)  (float),   A_i = n_b(k) - sum_{j <= i} counts_j,
 * on the market state (pass weight_dev as cva_regress_fit's W_dev): it learns the CVA given the
 * client's survival to t_i.  D_dev and counts_dev are [n+1][1][M] (n_cpty = 1); CVA_0 and the
 * other arguments as hsim_targets_cva (T_0 is the same, everyone is alive at t_0). */
int hsim_targets_alive(const hsim_grid* grid, int64_t M, int32_t n_b, const int32_t* n_b_per_block,
                       int32_t block_paths, int precision, const double* I_dev, const void* D_dev,
                       const int32_t* counts_dev, void* target_dev, float* weight_dev,
                       double* cva0_dev, void* workspace_dev, size_t ws_bytes, void* stream);

/* Intensity-based targets (Section 4.2, the intensity route eq:CVAint): the conditional
 * expectation of the inner average above given the outer path,
 *   T~_i = exp(I_i) sum_{j=i+1}^{n} sum_c D^c_j (exp(-Lambda^c_{j-1}) - exp(-Lambda^c_j)),
 * the minimal-variance regression target (no inner draws).  Lambda_dev [n+1][C][M] as written
 * by hsim_outer_paths; the rest as hsim_targets_cva (uniform weights, no n_b). */
int hsim_targets_intensity(const hsim_grid* grid, int32_t n_cpty, int64_t M, int precision,
                           const double* I_dev, const double* Lambda_dev, const void* D_dev,
                           void* target_dev, double* cva0_dev, void* workspace_dev, size_t ws_bytes,
                           void* stream);

/* The three stages above in one call: features_dev [n+1][d][M] (may be NULL),
 * target_dev [n+1][M], cva0_dev (one double).  The intermediate I, Lambda, D and counts
 * live in the workspace: hsim_workspace_bytes(HSIM_OP_FUSED, ...). */
int hsim_inner_defaults_cva(const hsim_market* market, const hsim_portfolio* book,
                            const hsim_grid* grid, uint64_t seed, int64_t path_begin, int64_t M,
                            int32_t n_b, const int32_t* n_b_per_block, int32_t block_paths,
                            int precision, int feature_mode, void* features_dev,
                            void* target_dev, double* cva0_dev, void* workspace_dev,
                            size_t ws_bytes, void* stream);

/* The whole simulation in one launch (Section 3.2's hierarchical sample, Appendix B, Section 4.2
 * eq:CVA_portfolio): outer paths, inner default draws and targets with the results of
 * hsim_outer_paths (features), hsim_inner_defaults and hsim_targets_cva bit for bit.  One
 * workgroup of 64 lanes per tile of 64 outer paths simulates them one lane per path (state in
 * registers) and writes, per path and date, the integer default thresholds of the rule
 * Lambda^c_j >= -log u, the exposures D^c_j and I_j into a path-major table in the workspace; the
 * same workgroup then draws each path's n_b x C inner defaults cooperatively (lanes = draws, the
 * default dates counted in an LDS histogram) and forms its targets.  I, Lambda, D and the counts
 * never reach the caller (hsim_inner_defaults_cva's date-major round trip), and the table is
 * about half their size.  Arguments as hsim_inner_defaults_cva (precision HSIM_FP32 or HSIM_FP64);
 * workspace hsim_workspace_bytes(HSIM_OP_FUSED_LAUNCH, ...).  HSIM_ERANGE when
 * (n+1) x n_cpty is too large for the kernel's LDS (more than 64 KiB: the separate stages then). */
int hsim_fused(const hsim_market* market, const hsim_portfolio* book, const hsim_grid* grid, uint64_t seed,
               int64_t path_begin, int64_t M, int32_t n_b, const int32_t* n_b_per_block, int32_t block_paths,
               int precision, int feature_mode, void* features_dev, void* target_dev, double* cva0_dev,
               void* workspace_dev, size_t ws_bytes, void* stream);

/* hsim_fused that also writes the forward states of the first n_keep paths (0 <= n_keep <= M)
 * date-major, as hsim_outer_paths writes them: I_dev [n+1][M], Lambda_dev [n+1][C][M] (double)
 * and D_dev [n+1][C][M] (float if FP32 else double), columns 0 .. n_keep - 1 written, the rest
 * untouched; with the features they are the input of cva_adjoint_forward (ld = M) for those
 * paths, so a solve needs no separate forward pass for its sensitivities.  The values equal
 * hsim_outer_paths' bit for bit.  n_keep = 0: hsim_fused (the three pointers may be NULL);
 * n_keep > 0 with a NULL pointer, or n_keep out of range: HSIM_EINVAL. */
int hsim_fused_keep(const hsim_market* market, const hsim_portfolio* book, const hsim_grid* grid, uint64_t seed,
                    int64_t path_begin, int64_t M, int32_t n_b, const int32_t* n_b_per_block, int32_t block_paths,
                    int precision, int feature_mode, void* features_dev, void* target_dev, double* cva0_dev,
                    int64_t n_keep, double* I_dev, double* Lambda_dev, void* D_dev, void* workspace_dev,
                    size_t ws_bytes, void* stream);

/* Pilot moments of the oversimulation chooser (Section 3.3, Proposition p:heurisN).  For
 * every date i and path k of T1_dev / T2_dev [n+1][M] (the n_b = 1 and n_b = 2 targets of
 * one seed, float if FP32 else double; with the common random numbers of
 * hsim_inner_defaults the first continuation of T2 is T1), the two pilot continuations
 * xi1 = T1, xi2 = 2 T2 - T1 give the pointwise losses g = (xi - phi)^2 against pred_dev
 * [n+1][M] (same type; NULL: phi = 0).  moments_dev [n+1][3] (double, device) receives
 * E[g], E[g^2] (both continuations pooled) and E[g g'], reduced in FP64 in a fixed order;
 * R = E[g g'] - E[g]^2 and Q = E[g^2] - E[g g'] give N*_i = sqrt(Q_i P / R_i) (e:optom). */
int hsim_oversim_moments(const hsim_grid* grid, int64_t M, int precision, const void* T1_dev,
                         const void* T2_dev, const void* pred_dev, double* moments_dev, void* stream);

/* Cost ratio of Section 3.3 (l:ratio): P, the cost of one outer path in units of one inner
 * continuation, from the times t and t_prime of two simulations with the same number of outer
 * paths and N, N_prime inner draws (t / t' = (P + N) / (P + N')):
 *   P = (t' N - t N') / (t - t').
 * Host arithmetic.  HSIM_EINVAL if a time is not positive, N == N_prime, t == t_prime, or P is not
 * positive and finite (timings that do not resolve the ratio). */
int hsim_oversim_cost_ratio(double t, double t_prime, double N, double N_prime, double* P_out);

/* Heuristic heur:MN of Section 3.3 from the pilot moments of hsim_oversim_moments (host copy,
 * [n_dates1][3]: E[g], E[g^2], E[g g'] per date): R_i = E[g g'] - E[g]^2,
 * Q_i = E[g^2] - E[g g'], N*_i = sqrt(Q_i P / R_i) (Proposition p:heurisN, e:optom) at every date
 * with R_i > 0 and Q_i >= 0 (NaN elsewhere, e.g. dates after the last maturity, which carry no
 * loss); N = the mean of the defined N*_i, at least 1 (1 if none is defined); M = Psi / (N + P)
 * outer paths for a budget of Psi inner-continuation units.  Host arrays R_out, Q_out, Nstar_out
 * [n_dates1] may be NULL.  Writes N and M; returns the number of dates with a defined N*_i, or
 * HSIM_EINVAL (P <= 0, Psi <= 0, n_dates1 < 1, NULL moments or outputs). */
int hsim_oversim_choose(int32_t n_dates1, const double* moments_host, double P, double Psi,
                        double* R_out, double* Q_out, double* Nstar_out, double* N_out, double* M_out);

/* Branched re-simulation (Section 3.3 twin Monte Carlo validation, e:val1/e:val2; the
 * nested Monte Carlo benchmark of Section 4.3 on eq:CVAint).  For every outer path k of
 * [path_begin, path_begin + M) and continuation b < n_branch (1 <= n_branch <= HSIM_MAX_BRANCH,
 * M * n_branch <= 2^31), the path is simulated exactly as hsim_outer_paths simulates it up to
 * the pricing date t_date (same Philox words and arithmetic), then with the branch words
 * (k, s, 16 b + (f >> 2), 3) after it, and
 *   xi_dev[b][k] = sum_{j > date} sum_c LGD_c exp(I_date - I_j) (MtM^c_j)^+
 *                  (exp(-Lambda^c_{j-1}) - exp(-Lambda^c_j))          (double, [n_branch][M]),
 * accumulated in FP64.  Given the state at t_date the samples of one path are independent
 * with conditional mean the CVA of eq:CVAint; 0 <= date <= n (date = n gives 0).  Market,
 * book and precision as hsim_outer_paths.  No workspace. */
int hsim_branch_cva(const hsim_market* market, const hsim_portfolio* book, const hsim_grid* grid,
                    uint64_t seed, int64_t path_begin, int64_t M, int32_t date, int32_t n_branch,
                    int precision, double* xi_dev, void* stream);

/* Nested and twin Monte Carlo errors of a prediction phi_dev [M] (float if FP32 else double;
 * NULL: phi = 0) against the continuation samples xi_dev [n_branch][M] of hsim_branch_cva,
 * n_branch >= 2.  With nu = mean_b xi and U = sum_{b != b'} xi_b xi_b' / (B (B-1)),
 * out_dev[6] (double, device) receives the path means, reduced in FP64 in a fixed order, of
 *   [0] nu  [1] nu^2  [2] U (unbiased for CVA^2)  [3] (phi - nu)^2 (nested error, biased by
 *   Var/B)  [4] phi^2 - 2 phi nu + U (twin error, unbiased for E[(phi - CVA)^2]; for B = 2
 *   exactly e:val1)  [5] phi.
 * The paper's relative error is sqrt(out[4] / out[2]).  Needs
 * hsim_workspace_bytes(HSIM_OP_BRANCH, NULL, NULL, M, precision) bytes of workspace. */
int hsim_branch_errors(int64_t M, int32_t n_branch, int precision, const void* phi_dev,
                       const double* xi_dev, double* out_dev, void* workspace_dev, size_t ws_bytes,
                       void* stream);

enum hsim_op { HSIM_OP_INNER = 1, HSIM_OP_TARGETS = 2, HSIM_OP_FUSED = 3, HSIM_OP_ADJOINT = 4,
               HSIM_OP_BRANCH = 5, HSIM_OP_FUSED_LAUNCH = 6 };

/* Device workspace (bytes) an operation needs for M paths and the given market/grid. */
size_t hsim_workspace_bytes(int op, const hsim_market* market, const hsim_grid* grid,
                            int64_t M, int precision);


/* ------------------------------------------------------------------------------------------
 * Regression of the targets on the market state (Section 2: NN^+ search space e:nnp,
 * BaseAlg = Algorithm 1, Backward learning = Algorithm 2).
 *
 * Network: `hidden` ReLU layers of `width` units and a linear output f; prediction
 * (f)^+ + mu.  Training of one date (BaseAlg with Adam): `epochs` epochs of contiguous
 * batches of `batch` rows; pos = 0 (no output ReLU) until epoch floor(epochs/2), at the end of
 * which the output layer is refitted in closed form with the hidden layers frozen and mu fixed
 * (the least-squares argmin of the pos = 0 loss: normal equations of [H 1] accumulated in FP64,
 * solved by a Cholesky factorisation in which a column with a zero diagonal or a pivot at or
 * below 1e-12 times its diagonal is linearly dependent on the columns before it and gets weight
 * 0, which leaves the fitted values those of the full least-squares problem), then pos = 1;
 * after every epoch the full-sample pos = 1 loss is computed and the best parameters are kept
 * (E = 1 therefore takes no refit).  Inputs are standardised per date (population mean and
 * standard deviation over the M rows) and targets divided by their root mean square; a date
 * whose targets are all zero is not trained and predicts 0.  Initial weights are
 * U(-1/sqrt(fan_in), 1/sqrt(fan_in)) from Philox words (layer, idx >> 2, init_tag, 2) with the
 * call's seed, biases and mu are 0.  Weights and activations are BF16 on the matrix cores with
 * FP32 accumulation; master weights, Adam moments, the output layer and the loss are FP32; the
 * refit is solved in FP64.
 * ------------------------------------------------------------------------------------------ */
typedef struct {
  int32_t hidden;     /* hidden layers; built shapes (width, hidden): (32,1) (32,2) (64,2) (128,2) (128,3) */
  int32_t width;      /* units per hidden layer */
  int32_t d_in;       /* inputs per row (the first d_in features of X): 1..32; up to 64 with
                         HSIM_REG_FP32 / HSIM_REG_FP64 (the model record then pads W_1 and the
                         scaling to 64 columns instead of 32) */
  int32_t epochs;     /* E >= 1 */
  int32_t batch;      /* rows per SGD batch; the last batch of an epoch may be shorter */
  double lr, beta1, beta2, eps; /* Adam (lr >= 0; lr = 0 leaves the network as initialised); the
                                   BF16 kernel uses them rounded to FP32 */
  int32_t warm_start; /* 0: every date trains independently from the same initial draw, all dates
                         in one persistent launch; 1: Backward learning, dates trained one after
                         another in the order given, each started from the previous date's result */
  int32_t init_tag;   /* Philox word selecting the initial draw */
  int32_t team;       /* workgroups training one date together (0..32); 0: chosen by the library
                         from the device size, the number of dates and the batch.  Results depend
                         on it only through the summation order of the batch gradient */
  int32_t dtype;      /* HSIM_REG_BF16: the matrix-core kernel described above (BF16 weights and
                         activations, FP32 accumulation), shapes as listed.  HSIM_REG_FP32 /
                         HSIM_REG_FP64: every product a rocBLAS GEMM / GEMV and every other step in
                         that precision (FP64 normal equations of the refit), dates trained one
                         after another (team ignored), any width 1..128 with 1..3 hidden layers;
                         X, Y, W, the model record and the loss history are then float (FP32) or
                         double (FP64).  Same initial draw, readings and record layout in all three */
  int32_t tile;       /* HSIM_REG_BF16: the kernels' wave tiling (0, 1, 2): the block of 16 x 16
                         output tiles each of the 8 waves owns at width 128 in the forward and
                         back-propagation products, 0: 2 units x 2 rows, 1: 4 x 1, 2: 1 x 4 (at
                         width 64: 2 x 1, 2 x 1, 1 x 2), and in the weight-gradient products 2 x 4,
                         4 x 2, 1 x 8 (out x in).  Picked by the autotuner; results depend on it only
                         through the summation order of the output unit's partial sums.  Ignored
                         (must be 0) by the FP32 / FP64 form */
} cva_mlp_cfg;

enum { HSIM_REG_BF16 = 0, HSIM_REG_FP32 = 1, HSIM_REG_FP64 = 2 };

/* Elements per date of the model array written by cva_regress_fit (parameters, then scaling); float
 * for HSIM_REG_BF16 / HSIM_REG_FP32, double for HSIM_REG_FP64. */
int cva_regress_record_floats(const cva_mlp_cfg* cfg);

/* Elements of the parameters at the head of a model record, in the order
 * W_1 [width][D] (columns >= d_in zero), b_1, W_2 [width][width], b_2, ..., W_hidden, b_hidden,
 * w_out [width], b_out, mu; the record continues with the input means [D], the inverse standard
 * deviations [D], the target scale and a trained flag.  D = 32 for d_in <= 32, else 64. */
int cva_regress_param_floats(const cva_mlp_cfg* cfg);

/* Device workspace for cva_regress_fit. */
size_t cva_regress_workspace_bytes(const cva_mlp_cfg* cfg, int32_t n_reg, int64_t M);

/* Fit one network per date j < n_reg on rows k < M of
 *   X_dev [n_dates_total][n_feat][M] (the features of hsim_outer_paths) and
 *   Y_dev [n_dates_total][M] (the targets of hsim_targets_cva),
 *   W_dev [n_dates_total][M] (row weights >= 0, or NULL for all 1: every loss becomes
 *   (1/rows) sum_k w_k (pred_k - y_k)^2 and the refit solves the weighted normal equations;
 *   with the weights of hsim_targets_alive this is the grouped form of the paper's
 *   per-inner-sample regression, Section 3.2),
 * date index dates[j] (host array).  model_dev [n_reg][cva_regress_record_floats] receives
 * the best parameters and the input scaling (BF16 form: 8-byte aligned, else HSIM_EINVAL); loss_hist_dev [n_reg][epochs] (may be NULL) the
 * full-sample loss after every epoch (in units of the scaled targets).  n_reg <= 512.
 * The team barriers and the loss helpers' waits are bounded: should one give up (it cannot while
 * every workgroup of the cooperative launch is resident), the fit stops early and the call
 * returns HSIM_ETIMEOUT.  Element type of X, Y, W, model and loss history: float, or double for
 * HSIM_REG_FP64.  Synchronous: returns once the fit on `stream` has completed. */
int cva_regress_fit(const cva_mlp_cfg* cfg, int32_t n_reg, const int32_t* dates, int32_t n_dates_total,
                    int64_t M, int32_t n_feat, const void* X_dev, const void* Y_dev,
                    const void* W_dev, uint64_t seed, void* model_dev, void* loss_hist_dev,
                    void* workspace_dev, size_t ws_bytes, void* stream);

/* Test hook: after a cva_regress_fit call with the same cfg, n_reg and M on this workspace, copy
 * each date's last parameters and Adam moments ([n_reg][n_params] each, float, or double for
 * HSIM_REG_FP64, the parameter order of the model record; any output may be NULL).  With
 * epochs = 1 and batch = M they hold one Adam step: m = (1 - beta1) g and v = (1 - beta2) g^2 of
 * the full-sample gradient g. */
int cva_regress_adam_state(const cva_mlp_cfg* cfg, int32_t n_reg, int64_t M, const void* workspace_dev,
                           size_t ws_bytes, void* params_dev, void* m_dev, void* v_dev, void* stream);

/* Test hook: the number of polls after which the regression's bounded waits give up (0 restores
 * the default, 2^22 polls of about a microsecond each).  Process-wide; affects later fits. */
int hsim_set_wait_limit(int32_t polls);

/* Predictions out_dev [n_reg][M] = ((f)^+ + mu) * y_scale of the fitted networks on X_dev (float,
 * or double for HSIM_REG_FP64, as the fit's); model_dev as the fit's (BF16 form: 8-byte aligned). */
int cva_regress_predict(const cva_mlp_cfg* cfg, int32_t n_reg, const int32_t* dates, int32_t n_dates_total,
                        int64_t M, int32_t n_feat, const void* X_dev, const void* model_dev,
                        void* out_dev, void* stream);


/* ------------------------------------------------------------------------------------------
 * Sensitivities of CVA_0.  The differentiated quantity is the smoothed estimator
 *   CVA_0 = (1/M) sum_k sum_c sum_{j=1}^{n} D^c_j (exp(-Lambda^c_{j-1}) - exp(-Lambda^c_j)),
 * the exact inner conditional expectation of the pathwise loss of eq:CVA_portfolio (its
 * indicator form is piecewise constant in the intensity integrals, so its pathwise derivative in
 * the credit parameters vanishes; Section 4.2 notes the intensity route is the minimal-variance
 * CVA learner).  Its expectation equals that of hsim_targets_cva's CVA_0.
 * Parameter order of grad_dev (hsim_n_params entries, 90 for 10 currencies / 8 counterparties):
 *   r0[n_ccy] fx0[n_ccy-1] lambda0[n_cpty] a[n_ccy] b[n_ccy] sigma_r[n_ccy] sigma_fx[n_ccy-1]
 *   kappa[n_cpty] theta[n_cpty] nu[n_cpty]
 * with the swap book's fixed rates held constant.  The forward sweep is the FP32 simulation of
 * hsim_outer_paths; credit parameters are differentiated by a forward-mode (tangent) sweep of the
 * CIR scheme, market parameters by a reverse sweep of the Vasicek / log-FX scheme that re-draws
 * the normals and inverts each Euler sub-step from the state stored at the next pricing date.
 * cva0_dev: one double; grad_dev: [hsim_n_params] doubles (device), or NULL for CVA_0 alone (the
 * reverse sweep is skipped).  With a gradient the credit sweep runs on a second stream of the
 * library's (one per device, default priority) forked from and joined back into `stream` by
 * events, beside the market sweep; results are ordered on `stream` as for any other call.
 * Workspace:
 * hsim_workspace_bytes(HSIM_OP_ADJOINT, ...).
 * ------------------------------------------------------------------------------------------ */
int hsim_n_params(const hsim_market* market);
int cva_adjoint(const hsim_market* market, const hsim_portfolio* book, const hsim_grid* grid, uint64_t seed,
                int64_t path_begin, int64_t M, double* cva0_dev, double* grad_dev, void* workspace_dev,
                size_t ws_bytes, void* stream);

/* cva_adjoint on outer paths that an earlier hsim_outer_paths call (same market, book, grid and
 * seed, FP32) has already simulated: their forward outputs are read from features_dev
 * [n+1][n_feat][ld] (the market factors first: any feature mode), I_dev [n+1][ld],
 * Lambda_dev [n+1][C][ld] and D_dev [n+1][C][ld], paths path_begin .. path_begin + M - 1 at
 * columns 0 .. M - 1 (ld >= M; e.g. the first M paths of a larger simulation), and no forward
 * pass is run.  The results equal cva_adjoint's.  The workspace (per-path gradient rows) may be
 * smaller than hsim_workspace_bytes(HSIM_OP_ADJOINT, ...): it needs (hsim_n_params + 1) * M
 * doubles, 256-byte aligned. */
int cva_adjoint_forward(const hsim_market* market, const hsim_portfolio* book, const hsim_grid* grid,
                        uint64_t seed, int64_t path_begin, int64_t M, int64_t ld, int32_t n_feat,
                        const float* features_dev, const double* I_dev, const double* Lambda_dev,
                        const float* D_dev, double* cva0_dev, double* grad_dev, void* workspace_dev,
                        size_t ws_bytes, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* HSIM_H */
