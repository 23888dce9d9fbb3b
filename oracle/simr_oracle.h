/*
 * simr_oracle.h -- plain FP64 CPU oracle for the Heston Monte Carlo / LSM hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists to check the GPU path; the
 * product never links, loads or calls it.  It shares no source with the GPU
 * library (no headers, helpers, constants or tables): every step is written
 * out again here, plainly, in double precision, in the order the method
 * states it.
 *
 * What it follows.  The paper (Klaisoongnoen et al., FPGA'24) names the stages
 * of its SIMR dataflow -- VariancePathQE, LogPricePathQE, AssetPathExponential,
 * longstaffSchwartzPathReduction, writeLongstaffSchwartzPath (Sec. 5, opening
 * paragraph) -- and the loop nest asset -> timestep -> path (Sec. 2.1 and
 * Listing 2), but never writes the equations.  The equations are taken from
 * the published methods those stage names refer to:
 *   - Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11) for the random words;
 *   - Box-Muller (1958) for the Gaussian transform;
 *   - Andersen (2008) Quadratic-Exponential scheme for variance and log-price;
 *   - full-truncation Euler (Lord, Koekkoek, van Dijk 2010) as the alternative;
 *   - Longstaff-Schwartz (2001) least-squares regression for early exercise;
 *   - pathwise derivatives (Giles, Glasserman 2006) for the Greeks, here in
 *     forward (tangent) mode.
 * The readings taken where the paper is silent are listed in the design notes.
 *
 * Conventions shared by every function below:
 *   dt = T/steps; states t_0..t_N with N = steps; x = ln(S/S0); v = variance.
 *   Random words for transition n (t_n -> t_{n+1}) of path p:
 *     counter = (n, p, stream, 0), key = (seed & 0xffffffff, seed >> 32).
 *   Words w0, w1 drive Box-Muller (Z1, Z2), w2 is the QE uniform U, w3 unused.
 *
 * Error behaviour: the functions assume validated inputs (they are test code);
 * they never allocate on behalf of the caller except internal scratch, which
 * they free before returning.  Return value 0 = success, -1 = allocation
 * failure or bad argument.
 */
#ifndef SIMR_ORACLE_H
#define SIMR_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { REF_EURO_CALL = 0, REF_EURO_PUT = 1, REF_AMER_PUT = 2, REF_AMER_CALL = 3 };
enum { REF_SCHEME_QE = 0, REF_SCHEME_FTE = 1, REF_SCHEME_QE_M = 2, REF_SCHEME_TG = 3, REF_SCHEME_BK = 4 };

typedef struct {
  double S0, K, T, r;
  double kappa, theta, xi, rho, v0;
  int32_t payoff;     /* REF_* payoff kind */
  int32_t steps;      /* N >= 1 */
  int64_t paths;      /* P >= 2 */
  uint64_t seed;      /* Philox key */
  uint32_t stream;    /* Philox counter word 2 */
  int32_t scheme;     /* REF_SCHEME_* */
} ref_option;

/* Philox4x32-10 block: 10 rounds on counter ctr[4] with key[2] -> out[4]. */
void ref_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);

/* The uniform on the 23-bit dyadic grid: ((w >> 9) + 1/2) * 2^-23, in (0,1). */
double ref_uniform(uint32_t w);

/* Box-Muller: z1 = sqrt(-2 ln u0) cos(2 pi u1), z2 = sqrt(-2 ln u0) sin(2 pi u1). */
void ref_box_muller(double u0, double u1, double* z1, double* z2);

/* One QE variance transition from v over dt (Andersen 2008, psi_c = 1.5);
 * z1 drives the quadratic branch, u the exponential branch. */
double ref_qe_variance_step(double v, double kappa, double theta, double xi, double dt,
                            double z1, double u);

/* One QE log-price transition (gamma1 = gamma2 = 1/2): returns x_{n+1}. */
double ref_qe_logprice_step(double x, double v, double vnext, double r, double kappa,
                            double theta, double xi, double rho, double dt, double z2);

/* Log of the moment-generating function of the QE variance transition from v,
 * ln E[exp(A V_{n+1}) | v_n = v], in the branch the variance step takes
 * (Andersen 2008, the martingale correction of the log-price scheme):
 *   quadratic branch, V = a (b + Z)^2:  A b^2 a / (1 - 2 A a) - ln(1 - 2 A a) / 2,
 *     defined for 2 A a < 1;
 *   exponential branch, V = 0 with probability p, else exponential of rate beta:
 *     ln(p + beta (1 - p) / (beta - A)), defined for A < beta;
 *   xi = 0 (deterministic V = m): A m.
 * *ok is set to 0 (and 0 returned) where the moment does not exist. */
double ref_qe_log_mgf(double v, double kappa, double theta, double xi, double dt, double A, int* ok);

/* One martingale-corrected QE log-price transition: the constant K0 is replaced by
 * K0* = -ln E[exp(A V_{n+1}) | v_n] - (K1 + K3 / 2) v_n with A = K2 + K4 / 2, so that
 * E[exp(x_{n+1} - x_n) | v_n] = exp(r dt) exactly; where the moment does not exist
 * the step keeps the uncorrected K0.  Returns x_{n+1}. */
double ref_qe_m_logprice_step(double x, double v, double vnext, double r, double kappa,
                              double theta, double xi, double rho, double dt, double z2);

/* Andersen's truncated Gaussian (TG) variance step: V = max(mu + sigma z1, 0) with mu = r sigma,
 * sigma = m / (r Phi(r) + phi(r)), where r = r(psi) makes the mean and variance of V those of
 * the CIR transition (m, s^2, psi = s^2 / m^2):
 *   ((r^2 + 1) Phi(r) + r phi(r)) / (r Phi(r) + phi(r))^2 = 1 + psi.
 * xi = 0 gives V = m.  The log-price step is QE's.  ref_tg_r returns r(psi) (psi > 0), solved
 * by safeguarded Newton iteration to FP64 rounding. */
double ref_tg_r(double psi);
double ref_tg_variance_step(double v, double kappa, double theta, double xi, double dt, double z1);

/* Broadie and Kaya's exact simulation of one step (REF_SCHEME_BK), from the uniforms of w2
 * and w3 and the normal z2 (z1 unused):
 *   V_t | v_u = c X, X noncentral chi-square with 4 kappa theta / xi^2 degrees of freedom and
 *     noncentrality v_u e^{-kappa dt} / c, c = xi^2 (1 - e^{-kappa dt}) / (4 kappa): inversion of
 *     its Poisson-mixture CDF at u_v (ref_bk_variance);
 *   I = integral of V over the step | v_u, V_t: inversion at u_i of the CDF obtained from the
 *     conditional characteristic function by the trapezoid Fourier sum
 *     F(x) = h x / pi + (2 / pi) sum_j sin(h j x) / j Re phi(h j), 2 pi / h = mu + 14 sd
 *     (ref_bk_integrated_variance; ref_bk_log_cf_re/_im give ln phi(a));
 *   x_t = x_u + r dt - I / 2 + rho (V_t - v_u - kappa theta dt + kappa I) / xi
 *         + sqrt((1 - rho^2) I) z2.
 * xi = 0: the deterministic CIR mean and its exact integral, rho taken as 0.  Roots are found
 * to ~1e-13 relative.  Greeks and baskets do not take this scheme. */
double ref_bk_variance(double v, double kappa, double theta, double xi, double dt, double u);
double ref_bk_integrated_variance(double vu, double vt, double kappa, double theta, double xi, double dt,
                                  double u);
double ref_bk_log_cf_re(double a, double vu, double vt, double kappa, double theta, double xi, double dt);
double ref_bk_log_cf_im(double a, double vu, double vt, double kappa, double theta, double xi, double dt);

/* One full-truncation Euler transition of (x, v). */
void ref_fte_step(double* x, double* v, double r, double kappa, double theta, double xi,
                  double rho, double dt, double z1, double z2);

/* Random words of paths [path0, path0+npaths) for steps [step0, step0+nsteps):
 * out[((p - path0) * nsteps + (n - step0)) * 4 + j]. */
void ref_rng_words(uint64_t seed, uint32_t stream, int64_t path0, int64_t npaths,
                   int32_t step0, int32_t nsteps, uint32_t* out);

/* Simulates paths [path0, path0+npaths) of the option to maturity.
 * Outputs (each may be NULL): xT (ln S_T/S0), vT (variance state at t_N),
 * disc_payoff (exp(-rT) * European payoff of the option's call/put kind).
 * nthreads >= 1 splits the paths; results do not depend on it. */
int ref_simulate(const ref_option* o, int64_t path0, int64_t npaths, int nthreads,
                 double* xT, double* vT, double* disc_payoff);

/* European price over paths [0, P): mean and standard error of the discounted
 * payoff.  sums[0] = sum X, sums[1] = sum X^2 (accumulated in path order). */
int ref_price_european(const ref_option* o, int nthreads, double* price, double* std_err,
                       double sums[2]);

/* Every path's state at every date (the path write-out of the LSM forward
 * pass): X[(n-1) * P + p] = x at t_n and V[...] = v at t_n for n = 1..N. */
int ref_path_states(const ref_option* o, int nthreads, double* X, double* V);

/* Least-squares solve of the 6x6 normal equations G beta = b by Cholesky with
 * diagonal pivoting; a column whose pivot falls to <= 1e-12 * max_i G_ii is
 * dropped (its coefficient set to 0).  Returns the number of kept columns. */
int ref_chol6_solve(const double G[36], const double b[6], double beta[6]);

/* American option by Longstaff-Schwartz over paths [0, P).
 *   price, std_err: the t_0 value max(h(S0), e^{-r dt} mean Y_1) and the SE of
 *   the Monte Carlo mean; tau (may be NULL, length P): exercise index in 1..N
 *   per path; exercised_at_t0: 1 when the intrinsic value won at t_0;
 *   lsm_flags: bit 0 set if some step had fewer than 6 in-the-money paths,
 *   bit 1 set if some regression dropped a column. */
int ref_price_american(const ref_option* o, int nthreads, double* price, double* std_err,
                       int32_t* tau, int32_t* exercised_at_t0, int32_t* lsm_flags);

/* The same, also writing the regression coefficients of every date n (basis
 * (1, a, a^2, c, a c, c^2)) to beta_out[n * 6 + i], n = 0..N (left untouched at
 * dates without a regression); beta_out may be NULL. */
int ref_price_american_beta(const ref_option* o, int nthreads, double* price, double* std_err,
                            int32_t* tau, int32_t* exercised_at_t0, int32_t* lsm_flags, double* beta_out);

/* Discounted cash flow e^{-r tau_p dt} h(S_{tau_p}) of every path p in [0, P)
 * stopped at the given index tau[p] in 0..N (0 = the intrinsic value at t_0). */
int ref_stopped_values(const ref_option* o, const int32_t* tau, int nthreads, double* out);

/* Pathwise Greeks by forward-mode (tangent) propagation in FP64, on the same
 * paths and branch choices as the pricing run (QE, FTE, martingale-corrected QE, whose K0* is
 * differentiated through the branch formula of the moment-generating function, and truncated
 * Gaussian, whose r(psi) is differentiated implicitly: dr/dpsi = A^3 / (2 (A^2 - B Phi)) with
 * A = r Phi + phi, B = (r^2 + 1) Phi + r phi; -1 for REF_SCHEME_BK).  grads[7] are d price / d
 * (S0, v0, theta, r, kappa, xi, rho); grad_se[7] their Monte Carlo standard
 * errors.  For American options the exercise times come from
 * ref_price_american on the same option and are held fixed.  price/std_err
 * are the pricing result. */
int ref_greeks(const ref_option* o, int nthreads, double* price, double* std_err,
               double grads[7], double grad_se[7]);

/* Pathwise Greeks with the stopping indices given: every path p is stopped at
 * tau[p] in 0..N and its discounted intrinsic value differentiated in forward
 * mode, the indices held fixed.  value/std_err are the mean of the stopped
 * cash flows and its standard error (the price of that exercise policy on these
 * paths).  Returns -1 on a NULL argument or an index outside 0..N. */
int ref_greeks_at_tau(const ref_option* o, const int32_t* tau, int nthreads, double* value, double* std_err,
                      double grads[7], double grad_se[7]);

/* The same two with two more sensitivities: grads[7] = d price / d T (N fixed, so the step
 * dt = T / N and every date move with T; exercise indices held fixed) and grads[8] = gamma,
 * d2 price / d S0^2, by the pathwise likelihood-ratio estimator: conditional on the variance
 * path, x at the stopping step is Gaussian in the asset variates z2_n with variance
 * sum sigma_n^2 (sigma_n the coefficient of z2_n in step n), so with W = sum sigma_n z2_n /
 * sum sigma_n^2 and xbar = dX / d ln S0 (pathwise), gamma = E[xbar (W - 1)] / S0^2.  Gamma is
 * NaN where some in-the-money path has sum sigma_n^2 = 0 (|rho| = 1), and for American options
 * and given stopping indices (the re-weighting would move each path's stopping decision onto
 * other trajectories); an option exercised at t_0 has gamma 0. */
int ref_greeks_ext(const ref_option* o, int nthreads, double* price, double* std_err,
                   double grads[9], double grad_se[9]);
int ref_greeks_at_tau_ext(const ref_option* o, const int32_t* tau, int nthreads, double* value, double* std_err,
                          double grads[9], double grad_se[9]);

/* ------------------------------------------------------------------------- */
/* Correlated baskets: d Heston assets, each with its own variance process and */
/* spot-variance correlation rho_i, whose independent asset drivers are       */
/* correlated across assets by the matrix C.                                  */
/*                                                                            */
/* Transition n of path p: asset i draws its words from the counter           */
/* (n, p, stream, i) -- so asset 0 draws exactly the single-asset words -- and */
/* takes (z1_i, z2_i) from Box-Muller and u_i from w2; the asset normals are   */
/* correlated, zc = L z2 with L L^T = C (lower Cholesky factor), and asset i   */
/* steps by its own scheme with (z1_i, zc_i, u_i) in place of (z1, z2, u).     */
/* The basket value is B = sum_i w_i S_i; payoffs are those of a single asset  */
/* with B in place of S.                                                       */
/* ------------------------------------------------------------------------- */
#define REF_MAX_ASSETS 32
#define REF_BASKET_NB 10 /* regression functions of the basket's Longstaff-Schwartz */

typedef struct {
  int32_t assets;  /* d, 1..REF_MAX_ASSETS */
  int32_t payoff;  /* REF_* payoff kind on the basket value */
  int32_t steps;   /* N >= 1 */
  int32_t scheme;  /* REF_SCHEME_* (every asset) */
  int64_t paths;   /* P >= 2 */
  uint64_t seed;
  uint32_t stream;
  uint32_t pad;
  double K, T, r;
  double w[REF_MAX_ASSETS], S0[REF_MAX_ASSETS], kappa[REF_MAX_ASSETS], theta[REF_MAX_ASSETS],
      xi[REF_MAX_ASSETS], rho[REF_MAX_ASSETS], v0[REF_MAX_ASSETS];
  double corr[REF_MAX_ASSETS * REF_MAX_ASSETS]; /* C, row-major, leading dimension REF_MAX_ASSETS */
} ref_basket;

/* Lower Cholesky factor of the d x d matrix C (both leading dimension REF_MAX_ASSETS);
 * -1 if C is not positive definite. */
int ref_corr_cholesky(int d, const double* C, double* L);

/* Terminal values of paths [path0, path0 + npaths): xT[i * d + k] = ln(S_T,k / S0_k),
 * vT[i * d + k] the variance of asset k, disc_payoff[i] = e^{-rT} h(B_T) (each may be NULL). */
int ref_basket_simulate(const ref_basket* b, int64_t path0, int64_t npaths, int nthreads, double* xT, double* vT,
                        double* disc_payoff);

/* European basket price over paths [0, P): mean and SE of the discounted payoff. */
int ref_basket_price_european(const ref_basket* b, int nthreads, double* price, double* std_err);

/* The basket's Longstaff-Schwartz write-out at dates n = 1..N:
 * X[(n-1) P + p] = ln(B_n / B_0), V[...] = sum_i w_i S_i,n max(v_i,n, 0) / B_n. */
int ref_basket_states(const ref_basket* b, int nthreads, double* X, double* V);

/* Least squares on nb x nb normal equations (nb <= 16, G row-major) by Cholesky with
 * diagonal pivoting, as ref_chol6_solve.  Returns the number of kept columns. */
int ref_chol_solve(int nb, const double* G, const double* bv, double* beta);

/* American basket option by Longstaff-Schwartz, regressing on the full cubic in
 * a = B/K - 1 and c = vbar/thetabar - 1 (vbar from ref_basket_states, thetabar =
 * sum w_i S0_i theta_i / B_0), basis (1, a, a^2, c, a c, c^2, a^3, a^2 c, a c^2, c^3);
 * otherwise as ref_price_american (flags bit 0: fewer than 10 in-the-money paths at some
 * date).  beta_out[n * 10 + i] as ref_price_american_beta (may be NULL). */
int ref_basket_price_american(const ref_basket* b, int nthreads, double* price, double* std_err, int32_t* tau,
                              int32_t* exercised_at_t0, int32_t* lsm_flags, double* beta_out);

/* Discounted stopped cash flows e^{-r tau_p dt} h(B_{tau_p}), tau[p] in 0..N. */
int ref_basket_stopped_values(const ref_basket* b, const int32_t* tau, int nthreads, double* out);

/* Basket Greeks in S0.  delta[i] = d price / d S0_i by the pathwise estimator
 * e^{-r tau dt} h'(B_tau) w_i S_tau,i / S0_i.  gamma[i * d + j] = d2 price / d S0_i d S0_j
 * (European options, tau NULL) by the pathwise-likelihood-ratio estimator: conditional on the
 * variance paths, the log-price increments of step n are Gaussian with covariance
 * diag(s_n) C diag(s_n) (s_nj the coefficient of zc_j), so a shift of ln S0_j spread over the
 * steps in proportion to s_nj^2 has the score W_j = sum_n s_nj u_nj / sum_n s_nj^2 with
 * u_n = L^{-T} z2_n, and with D_i the delta sample,
 *   gamma_ij = E[(D_i W_j / S0_j + D_j W_i / S0_i) / 2] - [i = j] E[D_i] / S0_i
 * (the symmetrised form).  Gamma is NaN for American options and given stopping indices,
 * and where a path with nonzero payoff slope has sum_n s_nj^2 = 0 (|rho_j| = 1).  With tau
 * NULL an American option is priced by ref_basket_price_american first and its exercise
 * indices held fixed (all 0 when exercised at t_0); price/std_err are then the LSM result,
 * else the mean of the (stopped) discounted cash flows. */
int ref_basket_greeks(const ref_basket* b, const int32_t* tau, int nthreads, double* price, double* std_err,
                      double* delta, double* delta_se, double* gamma, double* gamma_se);

/* Basket risk Greeks, every scheme but Broadie-Kaya.  vega_v0[i] = d price / d v0_i and
 * vega_theta[i] = d price / d theta_i by forward-mode pathwise tangents of asset i's own path
 * (its Heston parameters move no other asset), through the scheme's steps as ref_greeks does
 * for one option: e^{-r tau dt} h'(B_tau) w_i S_tau,i dx_i.  dcorr[i * d + j] (i != j,
 * symmetric; 0 on the diagonal) = d price / d C_ij with C_ij and C_ji moved together: the
 * correlated normals are zc = L z2, so with dL the derivative of the Cholesky factor in that
 * direction, dx_k = sum_n s_nk (dL z2_n)_k, s_nk the coefficient of zc_k in asset k's
 * increment of step n.  tau as for ref_basket_greeks (NULL: European at N, or an American
 * option's own Longstaff-Schwartz exercise indices, all 0 when exercised at t_0). */
int ref_basket_risk_greeks(const ref_basket* b, const int32_t* tau, int nthreads, double* price, double* std_err,
                           double* vega_v0, double* vega_v0_se, double* vega_theta, double* vega_theta_se,
                           double* dcorr, double* dcorr_se);

/* The Cholesky factor L of C and its derivative dL in the direction E_ij + E_ji (i != j), both
 * with leading dimension REF_MAX_ASSETS; -1 if C is not positive definite. */
int ref_corr_cholesky_tan(int d, const double* C, int i, int j, double* L, double* dL);

#ifdef __cplusplus
}
#endif
#endif
