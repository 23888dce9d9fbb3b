/*
 * simr.h -- C ABI of the MI355X (gfx950) Heston Monte Carlo / Longstaff-Schwartz
 * library: the hot path of the SIMR market-risk benchmark studied by
 * Klaisoongnoen et al., "Evaluating Versal AI Engines for option price
 * discovery in market risk analysis" (FPGA'24).
 *
 * The paper's problem statement (Sec. 2.1 and Sec. 3, Table 1) is a set of A
 * "assets" (options), each simulated over T time steps (252 per year) on P
 * paths; every (asset, step, path) element passes through the dataflow stages
 * VariancePathQE -> LogPricePathQE -> AssetPathExponential ->
 * longstaffSchwartzPathReduction -> writeLongstaffSchwartzPath (Sec. 5).
 * The arguments below follow that statement: one simr_option per asset, with
 * its steps and paths, plus the Heston and contract parameters.
 *
 * Conventions common to every entry point
 *   - Return value: simr_status, SIMR_OK (0) on success.  On any error the
 *     host outputs are left untouched and nothing has been launched unless the
 *     status is SIMR_EHIP; simr_last_error() gives a thread-local message.
 *   - Host pointers (option structs, result structs) are owned by the caller
 *     and only read/written during the call.
 *   - Device pointers (d_workspace, debug outputs) are owned by the caller;
 *     the library never frees caller memory.  Its only device allocation is
 *     the context's truncated Gaussian table (128 KiB), made by simr_create
 *     and freed by simr_destroy: no other call allocates or frees device
 *     memory.  Pinned host staging of the context (hipHostMalloc, a few KiB
 *     to a few MiB for the option tables and results) is allocated on first
 *     use and grows with the largest call; 64 bytes of it, for
 *     simr_price_noalloc, are allocated by simr_create.  Workspace size comes from
 *     simr_workspace_size(); its contents need no initialisation and are
 *     scratch between calls.
 *   - hip_stream is a hipStream_t (NULL = the default stream).  Work is
 *     enqueued on it in order; the calls that return host results synchronise
 *     that stream before writing them.  Calls on one context are not
 *     thread-safe with respect to each other.
 *   - Random numbers: Philox4x32-10 (Salmon et al., SC'11) with key
 *     (seed & 0xffffffff, seed >> 32) and counter (n, path, stream_id, 0) for
 *     the transition t_n -> t_{n+1}; words 0 and 1 give two normals by
 *     Box-Muller, word 2 the QE uniform, word 3 is unused.  A uniform is
 *     ((w >> 9) + 1/2) * 2^-23.  The same bits are drawn whatever the launch
 *     shape, so any path range can be re-run on its own.
 *   - Precision: path stepping in FP32; payoff sums Kahan-compensated in FP32
 *     per lane, then FP64 across lanes; Longstaff-Schwartz normal equations
 *     accumulated in FP32 per block, summed across blocks and solved in FP64.
 */
#ifndef SIMR_H
#define SIMR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  SIMR_OK = 0,
  SIMR_EINVAL = -1,        /* invalid argument (values, sizes, workspace too small) */
  SIMR_ENOMEM = -2,        /* host allocation failed inside the context */
  SIMR_EHIP = -3,          /* a HIP runtime call failed; see simr_last_error() */
  SIMR_EUNSUPPORTED = -4,  /* valid request that the library does not implement */
  SIMR_ENUMERIC = -5       /* a numerical failure detected on the device */
} simr_status;

/* Payoff kinds.  European options pay h(S_T) at maturity; American ones may be
 * exercised at any of the simulation dates t_1..t_N (and at t_0 through the
 * max with the intrinsic value), priced by Longstaff-Schwartz. */
typedef enum { SIMR_EURO_CALL = 0, SIMR_EURO_PUT = 1, SIMR_AMER_PUT = 2, SIMR_AMER_CALL = 3 } simr_payoff;

/* Discretisations: Andersen's Quadratic-Exponential scheme (the VariancePathQE /
 * LogPricePathQE stages of the paper), full-truncation Euler, QE with
 * Andersen's martingale correction (the log-price constant K0 replaced per step
 * by K0* = -ln E[exp(A V_{n+1}) | v_n] - (K1 + K3/2) v_n, A = K2 + K4/2, from the
 * moment-generating function of the QE variance transition, so that the
 * discounted asset price is an exact martingale; where that moment does not
 * exist the step keeps K0), or Andersen's truncated Gaussian variance step
 * (V = max(mu + sigma Z, 0) with mu and sigma matching the conditional mean m
 * and variance s^2 of the CIR transition; mu / m and sigma / m depend on
 * psi = s^2 / m^2 alone and are read from an 8192-point table in log2(psi) over
 * [2^-6, 2^14], solved in FP64 on the host by simr_create, held in device
 * memory of the context until simr_destroy, and interpolated linearly
 * (maximum relative error 1e-6); below 2^-6 the untruncated limit mu = m,
 * sigma = s is exact to 1e-14; above 2^14 the last entry holds) with QE's
 * log-price step.
 * SIMR_SCHEME_BK is Broadie and Kaya's exact simulation, in FP64 on the device (the FP32 path
 * state widened for each step): V_t | v_u from the noncentral chi-square law of the CIR
 * transition by inversion of its CDF at the uniform of Philox word 2; the integrated variance
 * I | v_u, V_t by inversion at the uniform of word 3 of the CDF given by the trapezoid Fourier
 * sum of its conditional characteristic function (the Bessel-bridge law; period twice
 * mean + 20 sd, Bessel series with a continuous phase); then
 * x_t = x_u + r dt - I/2 + rho (V_t - v_u - kappa theta dt + kappa I)/xi + sqrt((1 - rho^2) I) Z2.
 * It has no discretisation bias and costs about 1e6 FP64 operations per step: an accuracy
 * reference for few large steps (its Bessel series loses accuracy when
 * sqrt(v_u V_t) / (xi^2 dt) grows to the hundreds, i.e. at small steps).  Prices only:
 * Greeks and baskets return SIMR_EUNSUPPORTED. */
typedef enum {
  SIMR_SCHEME_QE = 0,
  SIMR_SCHEME_FTE = 1,
  SIMR_SCHEME_QE_M = 2,
  SIMR_SCHEME_TG = 3,
  SIMR_SCHEME_BK = 4
} simr_scheme;

/* One option ("asset" in the paper's Table 1).  Plain data, caller-owned. */
typedef struct {
  double S0, K, T, r;                  /* spot, strike, maturity (years), continuous rate */
  double kappa, theta, xi, rho, v0;    /* Heston: mean reversion, long variance, vol of vol,
                                          correlation, initial variance */
  int32_t payoff;                      /* simr_payoff */
  int32_t steps;                       /* N >= 1; dt = T / N */
  int64_t paths;                       /* 2 <= P <= 2^30 */
  uint64_t seed;                       /* Philox key */
  uint32_t stream_id;                  /* Philox counter word 2 */
  uint32_t reserved;                   /* must be 0 */
} simr_option;

/* Method parameters shared by all options of a call. */
typedef struct {
  int32_t scheme;            /* simr_scheme */
  int32_t checkpoint_every;  /* adjoint checkpoint interval in steps: 0 (= 16), 8, 16 or 32 */
  int32_t flags;             /* must be 0 */
  int32_t reserved;          /* must be 0 */
} simr_params;

/* Bits of simr_result.lsm_flags. */
#define SIMR_LSM_FEW_ITM 1       /* some date had fewer than 6 in-the-money paths: no exercise there */
#define SIMR_LSM_DROPPED 2       /* some regression dropped a collinear basis column */
#define SIMR_LSM_EXERCISE_T0 4   /* the intrinsic value at t_0 exceeded the continuation value */

typedef struct {
  double price;     /* Monte Carlo price */
  double std_err;   /* standard error of the Monte Carlo mean (0 if exercised at t_0) */
  int64_t paths;    /* paths used */
  int32_t lsm_flags;/* SIMR_LSM_* bits (American options) */
  int32_t reserved;
} simr_result;

/* Greeks are derivatives of the price with respect to, in this order:
 * S0 (delta), v0 (vega in v0), theta (vega in the long variance), r (rho),
 * kappa, xi, rho (the correlation). */
#define SIMR_NUM_GREEKS 7
typedef struct {
  double price, std_err;
  double g[SIMR_NUM_GREEKS];     /* pathwise adjoint Greeks */
  double g_se[SIMR_NUM_GREEKS];  /* their Monte Carlo standard errors */
  int32_t lsm_flags;
  int32_t reserved;
} simr_greeks_result;

/* The extended set: the 7 Greeks above, then
 *   g[7] = d price / d T with the step count N fixed (dt = T / N and every date move with T;
 *          American options hold their exercise indices fixed),
 *   g[8] = gamma, d2 price / d S0^2, European options only (NaN for American options, and when
 *          |rho| = 1): the pathwise likelihood-ratio estimator -- conditional on the variance
 *          path the log-price at maturity is Gaussian in the asset variates z2_n with variance
 *          sum sigma_n^2, so with W = sum sigma_n z2_n / sum sigma_n^2 and the pathwise
 *          derivative xbar = dX / d ln S0, gamma = E[xbar (W - 1)] / S0^2. */
#define SIMR_NUM_GREEKS_EXT 9
typedef struct {
  double price, std_err;
  double g[SIMR_NUM_GREEKS_EXT];
  double g_se[SIMR_NUM_GREEKS_EXT];
  int32_t lsm_flags;
  int32_t reserved;
} simr_greeks_ext_result;

typedef struct simr_ctx simr_ctx;  /* opaque: device properties, autotune cache, graph cache */

/* Creates a context bound to HIP device `device` (made current during calls).
 * Builds the truncated Gaussian table (host FP64 solves, then its 128 KiB of
 * device memory): the context's only device allocation.  Errors: SIMR_EINVAL
 * for a device index out of range, SIMR_EUNSUPPORTED for a device other than
 * gfx950, SIMR_EHIP when a HIP call fails; *ctx is written only on success. */
simr_status simr_create(simr_ctx** ctx, int device);
simr_status simr_destroy(simr_ctx* ctx);

/* Workspace bytes needed by op 0 = simr_price, 1 = simr_price_batch,
 * 2 = simr_greeks, 3 = simr_greeks_batch for the given options (n of them; n = 1
 * for ops 0 and 2; op 3 is the largest of: a European option's op-2 size, and a group of
 * consecutive American options' size, the groups taken in order as long as they stay within
 * 8 GiB or hold one option; any workspace from the largest single option's op-2 size up is
 * accepted by simr_greeks_batch).
 * Depends on the arguments only; ctx may be NULL.  Every entry point checks
 * its arguments before it needs the context, so argument errors are reported
 * as such even with ctx == NULL. */
simr_status simr_workspace_size(simr_ctx* ctx, int op, const simr_option* opts, int64_t n,
                                const simr_params* params, size_t* bytes);

/* Prices one option.  European: discounted payoff mean (the paper's stages up
 * to AssetPathExponential plus the discounted reduction).  American:
 * Longstaff-Schwartz backward induction over t_{N-1}..t_1 with the in-the-money
 * regression on {1, S, S^2, v, S v, v^2} (longstaffSchwartzPathReduction), the
 * path states written out once (writeLongstaffSchwartzPath). */
simr_status simr_price(simr_ctx* ctx, const simr_option* opt, const simr_params* params,
                       simr_result* out, void* d_workspace, size_t ws_bytes, void* hip_stream);

/* For callers that cannot allocate memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid allocation): simr_price for one
 * European option with no workspace argument and no allocation of any kind --
 * no hipMalloc, hipFree, hipHostMalloc or event creation.  Its device buffer
 * is a static array in the library's device code, one per GPU (2 MiB + 2 KiB,
 * held from the library's first use on that GPU until the process ends),
 * whose address simr_create records: the option record, the work-queue
 * counter (cleared by a kernel on every call), one {sum X, sum X^2} pair per
 * path tile and the result sums.  Limits: European options only (American
 * ones return SIMR_EUNSUPPORTED), and at most 131,072 path tiles, i.e.
 * 131,072 x (block x paths per lane) paths at the context's tile (33,554,432
 * at the untuned default 256 x 1); larger options return SIMR_EINVAL with
 * that limit in simr_last_error() before anything is launched.  The tile is
 * the one simr_price / simr_price_batch tuned on this context for the scheme,
 * or 256 x 1 if none was tuned (no timing runs here), so after such a call
 * the result equals simr_price's bit for bit.  Enqueues on hip_stream, copies
 * the two result sums into 64 bytes of pinned host memory that simr_create
 * allocated for this purpose (so the copy needs no staging) and synchronises
 * the stream.  Every call
 * on one GPU shares that GPU's array: calls that overlap on one GPU (other
 * threads, other contexts on the same device, or other streams) race and
 * must be serialised by the caller. */
simr_status simr_price_noalloc(simr_ctx* ctx, const simr_option* opt, const simr_params* params,
                               simr_result* out, void* hip_stream);

/* Prices n options of uneven strikes, maturities, step and path counts.
 * European options run in one persistent launch over (option, path-tile) work
 * units taken from an atomic queue in descending cost order; tile shape
 * chosen by the context's autotuner.  On a non-NULL hip_stream with
 * profiling off, that sequence (option table upload from pinned staging,
 * queue reset, persistent kernel, fixed-order finish, result download) is
 * captured into a hipGraph on the first call of each shape (European option
 * count, tile total, tile, scheme, grid, stream) and replayed by later calls
 * of that shape with the new options' contents; on the NULL stream, which
 * cannot be captured, or while profiling, the same launches are enqueued
 * directly (the results are the same bit for bit).  American
 * options are processed in passes of consecutive options (in the caller's
 * order) whose buffers fit 8 GiB together, or one alone if it needs more: the
 * forward passes and regression pre-passes of a pass run back to back, and
 * consecutive options with the same induction launch shape share one
 * cooperative launch, each on its own blocks, while their blocks fit
 * co-resident.  out[i] equals simr_price(opts[i]) on the same context bit for
 * bit.  The workspace size (simr_workspace_size, op 1) covers the largest
 * pass. */
simr_status simr_price_batch(simr_ctx* ctx, const simr_option* opts, int64_t n,
                             const simr_params* params, simr_result* out, void* d_workspace,
                             size_t ws_bytes, void* hip_stream);

/* Price plus the 7 pathwise Greeks of one option from one adjoint (reverse)
 * sweep per path, recomputing each segment of `checkpoint_every` steps from a
 * stored variance checkpoint with regenerated random numbers.  American
 * options hold the Longstaff-Schwartz exercise dates fixed.  QE, QE_M, FTE and TG schemes
 * (SIMR_EUNSUPPORTED for BK).  TG differentiates mu / m and sigma / m through a second table of
 * their exact FP64 derivatives in log2(psi) at the same nodes (a truncated step, V = 0, passes no
 * derivative; above the table, where the last entry holds, neither does psi).  QE_M differentiates the corrected constant
 * -ln E[exp(A V) | v] - (K1 + K3 / 2) v through A, the moments of the variance step and the
 * branch it takes; on steps where that moment does not exist the step's constant is the plain
 * C0 and its derivative is C0's (the jump of the constant where the moment stops existing is not
 * differentiated).  For FTE the derivative of sqrt(v+) at v+ = 0 is taken as 0, as is that of
 * sqrt(1 - rho^2) at |rho| = 1. */
simr_status simr_greeks(simr_ctx* ctx, const simr_option* opt, const simr_params* params,
                        simr_greeks_result* out, void* d_workspace, size_t ws_bytes, void* hip_stream);

/* simr_greeks plus d/dT and gamma (simr_greeks_ext_result) from the same sweep; the same
 * workspace (simr_workspace_size op 2), arguments and errors as simr_greeks. */
simr_status simr_greeks_ext(simr_ctx* ctx, const simr_option* opt, const simr_params* params,
                            simr_greeks_ext_result* out, void* d_workspace, size_t ws_bytes, void* hip_stream);

/* simr_greeks for n options: a risk run over many underlyings, the outer loop over assets of the
 * market-risk workload in the paper's Section 2.  The same results as n simr_greeks calls,
 * bit for bit, with one host synchronisation instead of n.  The options are enqueued one after
 * another on hip_stream and share the workspace (stream order keeps each option's kernels
 * behind the previous one's).  Consecutive American options whose buffers fit ws_bytes
 * together form groups: their path write-outs, Gram passes and backward inductions run as one
 * pass, the inductions side by side in one cooperative launch (simr_price_batch does the same),
 * then each option's adjoint; an option's induction sums in an order fixed by its own paths
 * per block, so grouping does not change its bits.  simr_workspace_size op 3 gives room for
 * groups of up to 8 GiB (two options of 2^20 paths x 252 steps fit one launch); any ws_bytes
 * from the largest single option's op-2 size up works, a smaller one making smaller groups.
 * Each option reads back into its own part of the context's pinned staging, which grows to a
 * few KiB per option.  out[i] (caller-owned, n entries) is written only when the
 * whole batch succeeds.  Errors: those of simr_greeks, with simr_last_error() naming the
 * first failing option; on a HIP failure mid-batch the stream is synchronised before the call
 * returns, so no read-back is left in flight. */
simr_status simr_greeks_batch(simr_ctx* ctx, const simr_option* opts, int64_t n, const simr_params* params,
                              simr_greeks_result* out, void* d_workspace, size_t ws_bytes, void* hip_stream);

/* ---- correlated baskets ------------------------------------------------------------------
 * The paper's asset dimension (Table 1: A assets, each with its own paths) read as correlated
 * underlyings of one basket.  Asset i follows its own Heston model (its own variance process,
 * spot-variance correlation rho_i and scheme step).  The asset drivers left after the
 * spot-variance correlation are correlated across assets by the d x d matrix C: in transition
 * n of path p, asset i draws the Philox words of counter (n, p, stream_id, i) -- asset 0 thus
 * draws exactly the words of a single option -- and the asset normals of the step become
 * zc = L z2 with L L^T = C (lower Cholesky factor, computed on the host in FP64).  With
 * xi_i = 0 the log-returns are correlated by C itself.  The payoff is that of simr_payoff on
 * the basket value B = sum_i w_i S_i.  American baskets are priced by Longstaff-Schwartz on
 * the basket's write-out (ln(B_n / B_0) and vbar_n = sum_i w_i S_i,n max(v_i,n, 0) / B_n per
 * path and date), regressing on the full cubic in a = B/K - 1 and c = vbar/thetabar - 1,
 * thetabar = sum_i w_i S0_i theta_i / B_0: (1, a, a^2, c, a c, c^2, a^3, a^2 c, a c^2, c^3),
 * a 10 x 10 Gram solved in FP64 per date (lsm_flags as for single options, the in-the-money
 * minimum being 10 paths).  The induction is one cooperative launch while the paths fit
 * co-resident (up to 4 per lane), else one launch per date on the same factors; the two
 * sum the right-hand sides in different groupings, so their prices agree to FP32 rounding of
 * those sums, not bit for bit. */
#define SIMR_MAX_ASSETS 32
#define SIMR_BASKET_NB 10

/* Plain data, caller-owned.  Per-asset arrays hold d = assets entries; corr is row-major with
 * leading dimension SIMR_MAX_ASSETS (corr[i * SIMR_MAX_ASSETS + j], i, j < d).  Entries beyond d
 * are ignored. */
typedef struct {
  int32_t assets;      /* d, 1 <= d <= SIMR_MAX_ASSETS */
  int32_t payoff;      /* simr_payoff on B */
  int32_t steps;       /* N >= 1 (as simr_option) */
  int32_t reserved0;   /* must be 0 */
  int64_t paths;       /* 2 <= P <= 2^30 (as simr_option) */
  uint64_t seed;       /* Philox key */
  uint32_t stream_id;  /* Philox counter word 2 */
  uint32_t reserved1;  /* must be 0 */
  double K, T, r;      /* strike on B, maturity, continuous rate */
  double w[SIMR_MAX_ASSETS];      /* weights w_i >= 0, sum_i w_i S0_i > 0 */
  double S0[SIMR_MAX_ASSETS];     /* per asset as simr_option: S0 > 0, kappa > 0, theta > 0, */
  double kappa[SIMR_MAX_ASSETS];  /* xi >= 0, |rho| <= 1, v0 >= 0 */
  double theta[SIMR_MAX_ASSETS];
  double xi[SIMR_MAX_ASSETS];
  double rho[SIMR_MAX_ASSETS];
  double v0[SIMR_MAX_ASSETS];
  double corr[SIMR_MAX_ASSETS * SIMR_MAX_ASSETS]; /* C: symmetric, unit diagonal, positive definite */
} simr_basket;

/* Price and the Greeks in the spots.  delta[i] = d price / d S0_i (pathwise:
 * e^{-r tau dt} h'(B_tau) w_i S_tau,i / S0_i).  gamma[i * SIMR_MAX_ASSETS + j] = d2 price /
 * d S0_i d S0_j, European baskets only, by the pathwise-likelihood-ratio estimator: conditional
 * on the variance paths the log-price increments of step n are Gaussian with covariance
 * diag(s_n) C diag(s_n) (s_nj the coefficient of zc_j in asset j's increment), so a shift of
 * ln S0_j spread over the steps in proportion to s_nj^2 has the score
 * W_j = sum_n s_nj u_nj / sum_n s_nj^2, u_n = L^{-T} z2_n, and with D_i the delta sample,
 *   gamma_ij = E[(D_i W_j / S0_j + D_j W_i / S0_i) / 2] - [i = j] E[D_i] / S0_i
 * (symmetric; a path whose D are all 0 contributes 0).  Gamma is NaN for American baskets
 * (the exercise indices of the Longstaff-Schwartz pass are held fixed for the deltas; an
 * option exercised at t_0 has delta_i = h'(B_0) w_i) and where a path with nonzero payoff
 * slope has sum_n s_nj^2 = 0 (|rho_j| = 1).  Entries beyond d are 0. */
typedef struct {
  double price, std_err;
  double delta[SIMR_MAX_ASSETS], delta_se[SIMR_MAX_ASSETS];
  double gamma[SIMR_MAX_ASSETS * SIMR_MAX_ASSETS], gamma_se[SIMR_MAX_ASSETS * SIMR_MAX_ASSETS];
  int32_t lsm_flags;
  int32_t reserved;
} simr_basket_greeks_result;

/* Risk Greeks of a basket: per-asset vegas and correlation sensitivities.
 *   vega_v0[i] = d price / d v0_i, vega_theta[i] = d price / d theta_i: forward-mode pathwise
 *     tangents of asset i's own path (its Heston parameters move no other asset) through the
 *     scheme's steps, times e^{-r tau dt} h'(B_tau) w_i S_tau,i.
 *   dcorr[i * SIMR_MAX_ASSETS + j] = d price / d C_ij with C_ij and C_ji moved together (i != j;
 *     symmetric, 0 on the diagonal): the correlated normals are zc = L z2, so with dL the
 *     derivative of the Cholesky factor in that direction (dL = L Phi(L^{-1} dC L^{-T}), Phi the
 *     lower triangle with half the diagonal) an asset's log-price moves by
 *     dx_k = sum_n s_nk (dL z2_n)_k, s_nk the coefficient of zc_k in its increment of step n.
 * Each with its Monte Carlo standard error; entries beyond d are 0.  American baskets hold the
 * exercise indices of their Longstaff-Schwartz pass fixed (price and lsm_flags are that pass's;
 * exercised at t_0, every risk Greek is 0). */
typedef struct {
  double price, std_err;
  double vega_v0[SIMR_MAX_ASSETS], vega_v0_se[SIMR_MAX_ASSETS];
  double vega_theta[SIMR_MAX_ASSETS], vega_theta_se[SIMR_MAX_ASSETS];
  double dcorr[SIMR_MAX_ASSETS * SIMR_MAX_ASSETS], dcorr_se[SIMR_MAX_ASSETS * SIMR_MAX_ASSETS];
  int32_t lsm_flags;
  int32_t reserved;
} simr_basket_risk_result;

/* Workspace bytes for op 0 = simr_basket_price (and the basket debug calls), 2 =
 * simr_basket_greeks, 3 = simr_basket_risk.  Depends on the arguments only; ctx may be NULL. */
simr_status simr_basket_workspace_size(simr_ctx* ctx, int op, const simr_basket* b, const simr_params* params,
                                       size_t* bytes);

/* Prices one basket (every scheme).  European: one launch over the paths (one path per lane,
 * every asset's state in registers), FP64 block sums.  American: the write-out, the Gram
 * pre-pass and the cooperative induction on the 10-function basis.  Synchronises hip_stream.
 * Errors: SIMR_EINVAL for invalid arguments (corr not symmetric with unit diagonal, or not
 * positive definite, included) before any launch; SIMR_EUNSUPPORTED for an American basket
 * whose paths do not fit co-resident (or with the per-date induction selected by
 * simr_set_lsm_launch). */
simr_status simr_basket_price(simr_ctx* ctx, const simr_basket* b, const simr_params* params, simr_result* out,
                              void* d_workspace, size_t ws_bytes, void* hip_stream);

/* Price, deltas and (European) cross-gammas of one basket (simr_basket_greeks_result), every
 * scheme, from one forward pass writing a record per path (discounted cash flow, delta
 * samples, scores) and FP64 moments over chunks of paths in a fixed order.  Same errors as
 * simr_basket_price.  Synchronises hip_stream. */
simr_status simr_basket_greeks(simr_ctx* ctx, const simr_basket* b, const simr_params* params,
                               simr_basket_greeks_result* out, void* d_workspace, size_t ws_bytes, void* hip_stream);

/* The basket risk Greeks (simr_basket_risk_result) from one forward pass with the tangents of
 * every asset's v0 and theta and the per-path sums s_nk z2_nm, writing one record per path (the
 * discounted cash flow, 2 d vega samples, d (d - 1) / 2 correlation samples), then FP64 sums over
 * chunks of paths in a fixed order.  Workspace: simr_basket_workspace_size op 3.  Errors:
 * SIMR_EINVAL as for simr_basket_price; SIMR_EUNSUPPORTED for more than 8 assets, or a scheme
 * other than QE, full-truncation Euler and the truncated Gaussian step.  Synchronises hip_stream. */
simr_status simr_basket_risk(simr_ctx* ctx, const simr_basket* b, const simr_params* params,
                             simr_basket_risk_result* out, void* d_workspace, size_t ws_bytes, void* hip_stream);

/* ---- test / debug entry points (same library) ------------------------------------------ */

/* Raw Philox words and the derived FP32 variates of paths [path0, path0+npaths),
 * steps [step0, step0+nsteps).  Device outputs, each optional (NULL):
 *   d_words[(p * nsteps + n) * 4 + j]  the 4 words,
 *   d_unif [(p * nsteps + n) * 3 + j]  the 3 uniforms,
 *   d_norm [(p * nsteps + n) * 2 + j]  Z1, Z2 (Box-Muller).
 * Asynchronous on hip_stream. */
simr_status simr_debug_draws(simr_ctx* ctx, uint64_t seed, uint32_t stream_id, int64_t path0,
                             int64_t npaths, int32_t step0, int32_t nsteps, uint32_t* d_words,
                             float* d_unif, float* d_norm, void* hip_stream);

/* Per-path terminal values of one option with the production path code:
 * d_xT[p] = ln(S_T/S0), d_vT[p] = variance state at t_N, d_payoff[p] = the
 * discounted European payoff (call or put by the option's kind).  Device
 * outputs of opt->paths floats each, each optional.  Asynchronous. */
simr_status simr_debug_paths(simr_ctx* ctx, const simr_option* opt, const simr_params* params,
                             float* d_xT, float* d_vT, float* d_payoff, void* hip_stream);

/* American option: the price (as simr_price) plus the exercise index of every
 * path (d_tau[p] in 1..N, device, opt->paths int32) and the FP64 regression
 * coefficients of every date (d_beta[n * 6 + i], n = 0..N, zero where no
 * regression ran; basis (1, a, a^2, c, a c, c^2), a = S/K - 1,
 * c = v/theta - 1).  Synchronises hip_stream. */
simr_status simr_debug_lsm(simr_ctx* ctx, const simr_option* opt, const simr_params* params,
                           simr_result* out, int32_t* d_tau, double* d_beta, void* d_workspace,
                           size_t ws_bytes, void* hip_stream);

/* Per-path terminal values of one basket with the production path code: d_xT[p * d + i] =
 * ln(S_T,i / S0_i), d_vT[p * d + i] = variance of asset i at t_N, d_payoff[p] = the
 * discounted European payoff on B_T.  Device outputs (each optional), a workspace of
 * simr_basket_workspace_size op 0.  Synchronises hip_stream. */
simr_status simr_debug_basket_paths(simr_ctx* ctx, const simr_basket* b, const simr_params* params, float* d_xT,
                                    float* d_vT, float* d_payoff, void* d_workspace, size_t ws_bytes,
                                    void* hip_stream);

/* American basket: the price (as simr_basket_price) plus every path's exercise index (d_tau[p]
 * in 1..N) and the FP64 coefficients of every date (d_beta[n * 10 + i], n = 0..N, zero where no
 * regression ran), basis as above.  Synchronises hip_stream. */
simr_status simr_debug_basket_lsm(simr_ctx* ctx, const simr_basket* b, const simr_params* params, simr_result* out,
                                  int32_t* d_tau, double* d_beta, void* d_workspace, size_t ws_bytes,
                                  void* hip_stream);

/* Launch shape of the Longstaff-Schwartz backward induction.  mode 0 (default):
 * one cooperative persistent launch for all dates, the lanes keeping their
 * paths' cash flows in registers and the blocks exchanging their sums once
 * per date through tagged words, on at most grid_max blocks (0 keeps the
 * current value, initially 64; capped at 256); falls back to mode 1 when the paths do not fit co-resident.
 * mode 1: one launch per date, the last block to finish solving the
 * regression.  Both give the same prices up to FP32 summation order.
 * mode 2 (a test of failure handling): as mode 0, but the exchange's status word is set
 * before each cooperative induction, as a timed-out wait would set it; every wait of the
 * induction then gives up at once, the launch completes, and the call returns SIMR_ENUMERIC
 * ("Longstaff-Schwartz exchange wait timed out").  The next call in mode 0 runs normally.
 * modes 3 and 4: as mode 0, with every cooperative launch of single-asset options on 256-thread
 * blocks (four times the paths per lane) or on 1024-thread blocks; mode 0 takes per launch the
 * size that holds more options co-resident (two options of 2^20 paths fit one launch only on
 * 256-thread blocks).  An option's paths per block, not the block size, fix its summation
 * order, so modes 0, 3 and 4 give the same bits. */
simr_status simr_set_lsm_launch(simr_ctx* ctx, int32_t mode, int32_t grid_max);

/* Host-side fault injection, a test of the error paths (no kernel is affected).  Arms the
 * context so that its nth HIP call (nth >= 1, counted from this call) of one kind reports a
 * failure: kind 1 = allocations (hipMalloc, hipHostMalloc, hipEventCreate), 2 = launches
 * (kernels and graph launches), 3 = copies and synchronisations; kind 0 disarms.  An
 * allocation or launch that fails this way is not made; a copy or synchronisation is made and
 * then reported as failed, so no work of the failing call is left running behind the error.
 * The call that meets the fault returns SIMR_EHIP ("injected ... failure" in
 * simr_last_error()) with its host outputs untouched, and the plan disarms itself; later calls
 * run normally.  *fired (optional) receives the number of faults injected on this context
 * before this call.  The environment variable SIMR_FAULT_INJECT="kind[:nth]" (kind alloc,
 * launch, sync, or create: simr_create itself returns SIMR_EHIP before any HIP call) arms every
 * new context the same way; any other value makes simr_create return SIMR_EINVAL. */
simr_status simr_debug_fault(simr_ctx* ctx, int32_t kind, int32_t nth, int64_t* fired);

/* Batch graphs of this context: how many were captured, and how many launches
 * of a captured graph (the first launch after each capture included) ran. */
simr_status simr_debug_graph_stats(simr_ctx* ctx, int64_t* captures, int64_t* launches);

/* Autotuner control: the tile shape (block size, paths per lane) the batch
 * kernel uses; chosen by timing candidates on first use unless set here. */
simr_status simr_get_tile(simr_ctx* ctx, int32_t* block, int32_t* paths_per_lane);
simr_status simr_set_tile(simr_ctx* ctx, int32_t block, int32_t paths_per_lane);

/* Profiling: while enabled, the library records HIP events on the call's
 * stream around each launch of the groups below (the Longstaff-Schwartz induction
 * in one-launch-per-date mode: around all dates of an option) and accumulates
 * their durations and count (the batch graph is not used while profiling, so
 * every launch is bracketed).  A cooperative induction launch may carry several
 * options.  simr_profile_read waits for the recorded events. */
#define SIMR_PROF_PRICE 0    /* persistent European pricing kernel (simr_price / simr_price_batch) */
#define SIMR_PROF_SPILL 1    /* forward pass writing the path states (American options) */
#define SIMR_PROF_LSM 2      /* Longstaff-Schwartz backward induction over all dates */
#define SIMR_PROF_CKPT 3     /* forward pass writing variance checkpoints (European Greeks) */
#define SIMR_PROF_ADJOINT 4  /* adjoint reverse sweep */
#define SIMR_PROF_GRAM 5     /* Gram and right-hand-side sums of all dates (before the induction) */
#define SIMR_PROF_FACTOR 6   /* FP64 factorisations of those sums, all dates */
#define SIMR_PROF_GROUPS 7
simr_status simr_profile_enable(simr_ctx* ctx, int on);
/* Which groups profiling records: bit g of mask for group g (default: all groups).  Each
 * recorded launch adds two events to the stream, so recording only the group being measured
 * keeps the others' launches as they run unprofiled.  SIMR_EINVAL for a zero mask or bits
 * beyond the groups. */
simr_status simr_profile_groups(simr_ctx* ctx, uint32_t mask);
simr_status simr_profile_read(simr_ctx* ctx, int group, double* total_ms, int64_t* launches);
simr_status simr_profile_reset(simr_ctx* ctx);

const char* simr_status_string(simr_status s);
const char* simr_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* SIMR_H */
