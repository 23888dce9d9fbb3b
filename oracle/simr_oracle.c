/*
 * simr_oracle.c -- plain FP64 CPU oracle (TEST INFRASTRUCTURE ONLY).
 *
 * Only the test suite, the smoke check and the benchmark's CPU-baseline leg
 * use this library; the GPU product never links or calls it, and the two share
 * no source.  Everything here is double precision, computed in the order the
 * method states it, with no blocking, fusion or reordering.  Build flags:
 * -O2 -ffp-contract=off (no fused multiply-adds, no fast-math), so that every
 * operation is the IEEE double operation written in the source.
 *
 * Method sources (the paper names the stages but not their equations; see the
 * header for the published methods each stage refers to):
 *   Philox4x32-10 ............ Salmon et al., SC'11, Sec. 3-4 (round function,
 *                              Weyl key schedule, multipliers).
 *   Uniform map, Box-Muller .. readings of the paper's "two data points per
 *                              element" (Sec. 3, Table 1) as in-kernel draws.
 *   VariancePathQE ........... Andersen (2008), QE scheme: moment matching of
 *                              the CIR transition, quadratic branch for
 *                              psi <= psi_c, exponential branch otherwise.
 *   LogPricePathQE ........... Andersen (2008), log-price discretisation with
 *                              K0..K4 and trapezoidal gamma1 = gamma2 = 1/2.
 *                              Truncated Gaussian variant (scheme TG):
 *                              V = max(mu + sigma Z, 0) moment-matched.
 *                              Martingale-corrected variant (scheme QE_M):
 *                              K0 replaced by K0* from the moment-generating
 *                              function of the QE variance transition.
 *   AssetPathExponential ..... S = S0 exp(x).
 *   longstaffSchwartzPathReduction / writeLongstaffSchwartzPath
 *                          ... Longstaff-Schwartz (2001): backward induction,
 *                              in-the-money regression on {1,S,S^2,v,Sv,v^2}.
 *   Greeks ................... pathwise derivatives (Giles-Glasserman 2006) in
 *                              forward mode, 7 tangent directions.
 */
#include "simr_oracle.h"

#include <complex.h>
#include <math.h>
#include <pthread.h>
#include <stdlib.h>
#include <string.h>

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

/* ------------------------------------------------------------------------- */
/* Philox4x32-10 (Salmon et al. 2011).                                        */
/* ------------------------------------------------------------------------- */

/* Multipliers and Weyl key increments of Philox4x32 as published. */
static const uint32_t PHILOX_MUL_A = 0xD2511F53u;
static const uint32_t PHILOX_MUL_B = 0xCD9E8D57u;
static const uint32_t PHILOX_WEYL_A = 0x9E3779B9u;
static const uint32_t PHILOX_WEYL_B = 0xBB67AE85u;

/* One round: two 32x32 -> 64-bit products, then the S-box/P-box mix
 * (c0, c1, c2, c3) -> (hi(B*c2) ^ c1 ^ k0, lo(B*c2), hi(A*c0) ^ c3 ^ k1, lo(A*c0)). */
static void philox_round(uint32_t c[4], const uint32_t k[2]) {
  uint64_t prodA = (uint64_t)PHILOX_MUL_A * (uint64_t)c[0];
  uint64_t prodB = (uint64_t)PHILOX_MUL_B * (uint64_t)c[2];
  uint32_t hiA = (uint32_t)(prodA >> 32), loA = (uint32_t)prodA;
  uint32_t hiB = (uint32_t)(prodB >> 32), loB = (uint32_t)prodB;
  uint32_t n0 = hiB ^ c[1] ^ k[0];
  uint32_t n1 = loB;
  uint32_t n2 = hiA ^ c[3] ^ k[1];
  uint32_t n3 = loA;
  c[0] = n0;
  c[1] = n1;
  c[2] = n2;
  c[3] = n3;
}

void ref_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  uint32_t c[4] = {ctr[0], ctr[1], ctr[2], ctr[3]};
  uint32_t k[2] = {key[0], key[1]};
  for (int round = 0; round < 10; ++round) {
    if (round > 0) { /* the key is bumped between rounds, not before the first */
      k[0] += PHILOX_WEYL_A;
      k[1] += PHILOX_WEYL_B;
    }
    philox_round(c, k);
  }
  for (int j = 0; j < 4; ++j) out[j] = c[j];
}

/* ------------------------------------------------------------------------- */
/* Uniform map and Gaussian transform.                                        */
/* ------------------------------------------------------------------------- */

double ref_uniform(uint32_t w) {
  /* top 23 bits, centred in their cell: the odd multiples of 2^-24 in (0,1) */
  return ((double)(w >> 9) + 0.5) * 0x1p-23;
}

void ref_box_muller(double u0, double u1, double* z1, double* z2) {
  double radius = sqrt(-2.0 * log(u0));
  double angle = 2.0 * M_PI * u1;
  *z1 = radius * cos(angle);
  *z2 = radius * sin(angle);
}

/* ------------------------------------------------------------------------- */
/* Heston discretisations.                                                    */
/* ------------------------------------------------------------------------- */

static const double PSI_C = 1.5;   /* QE switching level psi_c (Andersen's choice) */
static const double GAMMA1 = 0.5;  /* trapezoidal weights of the variance integral */
static const double GAMMA2 = 0.5;

/* CIR conditional moments over dt, as the QE scheme matches them:
 *   E[v(t+dt) | v] = theta + (v - theta) e^{-kappa dt}
 *   Var[v(t+dt) | v] = v xi^2 e^{-kappa dt}(1 - e^{-kappa dt})/kappa
 *                    + theta xi^2 (1 - e^{-kappa dt})^2 / (2 kappa)        */
double ref_qe_variance_step(double v, double kappa, double theta, double xi, double dt,
                            double z1, double u) {
  double E = exp(kappa * -dt);
  double omE = 1.0 - E;
  double m = theta + (v - theta) * E;
  double s2 = v * (((xi * xi) * E) * omE / kappa) + ((theta * (xi * xi)) * (omE * omE)) / (2.0 * kappa);
  if (!(s2 > 0.0)) return m; /* xi = 0: the variance moves deterministically */
  double psi = s2 / (m * m);
  if (psi <= PSI_C) {
    /* quadratic branch: V = a (b + Z)^2 with E[V] = m, Var[V] = s2 */
    double t = 2.0 / psi;
    double b2 = (t - 1.0) + sqrt(t) * sqrt(t - 1.0);
    double b = sqrt(b2);
    double a = m / (1.0 + b2);
    double bz = b + z1;
    return a * (bz * bz);
  }
  /* exponential branch: mass p at zero, exponential tail of rate beta */
  double p = (psi - 1.0) / (psi + 1.0);
  double beta = (1.0 - p) / m;
  if (u <= p) return 0.0;
  return log((1.0 - p) / (1.0 - u)) / beta;
}

/* The K coefficients of the QE log-price update.  With xi = 0 the variance is
 * deterministic and the rho/xi terms (which carry the part of the asset noise
 * correlated with the variance noise) are absent: rho is taken as 0. */
static void qe_k_coeffs(double kappa, double theta, double xi, double rho, double dt, double K[5]) {
  double rh = (xi > 0.0) ? rho : 0.0;
  double rox = (xi > 0.0) ? rh / xi : 0.0;
  K[0] = (xi > 0.0) ? -((rh * kappa) * theta * dt) / xi : 0.0;
  K[1] = GAMMA1 * dt * (kappa * rox - 0.5) - rox;
  K[2] = GAMMA2 * dt * (kappa * rox - 0.5) + rox;
  K[3] = GAMMA1 * dt * (1.0 - rh * rh);
  K[4] = GAMMA2 * dt * (1.0 - rh * rh);
}

double ref_qe_logprice_step(double x, double v, double vnext, double r, double kappa,
                            double theta, double xi, double rho, double dt, double z2) {
  double K[5];
  qe_k_coeffs(kappa, theta, xi, rho, dt, K);
  double w = K[3] * v + K[4] * vnext;
  return x + r * dt + K[0] + K[1] * v + K[2] * vnext + sqrt(w) * z2;
}

double ref_qe_log_mgf(double v, double kappa, double theta, double xi, double dt, double A, int* ok) {
  /* the same conditional moments and branch choice as ref_qe_variance_step */
  double E = exp(kappa * -dt);
  double omE = 1.0 - E;
  double m = theta + (v - theta) * E;
  double s2 = v * (((xi * xi) * E) * omE / kappa) + ((theta * (xi * xi)) * (omE * omE)) / (2.0 * kappa);
  *ok = 1;
  if (!(s2 > 0.0)) return A * m;
  double psi = s2 / (m * m);
  if (psi <= PSI_C) {
    double t = 2.0 / psi;
    double b2 = (t - 1.0) + sqrt(t) * sqrt(t - 1.0);
    double a = m / (1.0 + b2);
    double d = 1.0 - 2.0 * A * a;
    if (!(d > 0.0)) { *ok = 0; return 0.0; }
    /* E[exp(A a (b + Z)^2)] = exp(A a b^2 / d) / sqrt(d) for Z ~ N(0, 1) */
    return A * b2 * a / d - 0.5 * log(d);
  }
  double p = (psi - 1.0) / (psi + 1.0);
  double beta = (1.0 - p) / m;
  if (!(A < beta)) { *ok = 0; return 0.0; }
  /* E[exp(A V)] = p + (1 - p) beta / (beta - A) */
  return log(p + beta * (1.0 - p) / (beta - A));
}

double ref_qe_m_logprice_step(double x, double v, double vnext, double r, double kappa,
                              double theta, double xi, double rho, double dt, double z2) {
  double K[5];
  qe_k_coeffs(kappa, theta, xi, rho, dt, K);
  double A = K[2] + 0.5 * K[4];
  int ok;
  double lm = ref_qe_log_mgf(v, kappa, theta, xi, dt, A, &ok);
  double k0 = ok ? -lm - (K[1] + 0.5 * K[3]) * v : K[0];
  double w = K[3] * v + K[4] * vnext;
  return x + r * dt + k0 + K[1] * v + K[2] * vnext + sqrt(w) * z2;
}

static double std_pdf(double x) { return exp(-0.5 * x * x) / sqrt(2.0 * M_PI); }
static double std_cdf(double x) { return 0.5 * erfc(-x / sqrt(2.0)); }

/* g(r) = ((r^2 + 1) Phi + r phi) / (r Phi + phi)^2 - 1: the squared coefficient of variation
 * of max(r + Z, 0); it falls monotonically from infinity (r -> -inf) to 0 (r -> +inf). */
static double tg_cv2(double r) {
  double P = std_cdf(r), f = std_pdf(r);
  double m1 = r * P + f;
  return ((r * r + 1.0) * P + r * f) / (m1 * m1) - 1.0;
}

double ref_tg_r(double psi) {
  if (!(psi > 0.0)) return INFINITY;
  /* bracket: tg_cv2 is decreasing in r */
  double lo = -1.0, hi = 1.0;
  while (tg_cv2(lo) < psi) lo *= 2.0;
  while (tg_cv2(hi) > psi) hi *= 2.0;
  for (int it = 0; it < 200; ++it) {
    double mid = 0.5 * (lo + hi);
    if (mid == lo || mid == hi) break;
    if (tg_cv2(mid) > psi) lo = mid; else hi = mid;
  }
  return 0.5 * (lo + hi);
}

double ref_tg_variance_step(double v, double kappa, double theta, double xi, double dt, double z1) {
  double E = exp(kappa * -dt);
  double omE = 1.0 - E;
  double m = theta + (v - theta) * E;
  double s2 = v * (((xi * xi) * E) * omE / kappa) + ((theta * (xi * xi)) * (omE * omE)) / (2.0 * kappa);
  if (!(s2 > 0.0)) return m; /* xi = 0: the variance moves deterministically */
  double psi = s2 / (m * m);
  double r = ref_tg_r(psi);
  double sigma = m / (r * std_cdf(r) + std_pdf(r));
  double V = r * sigma + sigma * z1;
  return V > 0.0 ? V : 0.0;
}

void ref_fte_step(double* x, double* v, double r, double kappa, double theta, double xi,
                  double rho, double dt, double z1, double z2) {
  double vp = (*v > 0.0) ? *v : 0.0;
  double sq = sqrt(vp * dt);
  double zs = rho * z1 + sqrt(1.0 - rho * rho) * z2;
  double vn = *v + kappa * (theta - vp) * dt + xi * sq * z1;
  *x = *x + (r - 0.5 * vp) * dt + sq * zs;
  *v = vn;
}

/* ------------------------------------------------------------------------- */
/* Paths.                                                                     */
/* ------------------------------------------------------------------------- */

static void words_of(const ref_option* o, int64_t path, int32_t step, uint32_t w[4]) {
  uint32_t ctr[4] = {(uint32_t)step, (uint32_t)path, o->stream, 0u};
  uint32_t key[2] = {(uint32_t)(o->seed & 0xffffffffu), (uint32_t)(o->seed >> 32)};
  ref_philox4x32_10(ctr, key, w);
}

void ref_rng_words(uint64_t seed, uint32_t stream, int64_t path0, int64_t npaths,
                   int32_t step0, int32_t nsteps, uint32_t* out) {
  ref_option o;
  memset(&o, 0, sizeof o);
  o.seed = seed;
  o.stream = stream;
  for (int64_t p = 0; p < npaths; ++p)
    for (int32_t n = 0; n < nsteps; ++n) words_of(&o, path0 + p, step0 + n, out + ((size_t)p * nsteps + n) * 4);
}

/* The three driving variates of transition n of a path. */
static void draws_of(const ref_option* o, int64_t path, int32_t n, double* z1, double* z2, double* u, double* u2) {
  uint32_t w[4];
  words_of(o, path, n, w);
  ref_box_muller(ref_uniform(w[0]), ref_uniform(w[1]), z1, z2);
  *u = ref_uniform(w[2]);
  *u2 = ref_uniform(w[3]);
}

void ref_bk_step(double* x, double* v, double r, double kappa, double theta, double xi, double rho, double dt,
                 double z2, double u_v, double u_i);

/* u2 (from w3) is used by the Broadie-Kaya scheme only: it draws the integrated variance. */
static void transition(const ref_option* o, double dt, double* x, double* v, double z1, double z2, double u,
                       double u2) {
  if (o->scheme == REF_SCHEME_BK) {
    ref_bk_step(x, v, o->r, o->kappa, o->theta, o->xi, o->rho, dt, z2, u, u2);
  } else if (o->scheme == REF_SCHEME_FTE) {
    ref_fte_step(x, v, o->r, o->kappa, o->theta, o->xi, o->rho, dt, z1, z2);
  } else {
    double vn = (o->scheme == REF_SCHEME_TG) ? ref_tg_variance_step(*v, o->kappa, o->theta, o->xi, dt, z1)
                                             : ref_qe_variance_step(*v, o->kappa, o->theta, o->xi, dt, z1, u);
    if (o->scheme == REF_SCHEME_QE_M)
      *x = ref_qe_m_logprice_step(*x, *v, vn, o->r, o->kappa, o->theta, o->xi, o->rho, dt, z2);
    else
      *x = ref_qe_logprice_step(*x, *v, vn, o->r, o->kappa, o->theta, o->xi, o->rho, dt, z2);
    *v = vn;
  }
}

static int is_call(int payoff) { return payoff == REF_EURO_CALL || payoff == REF_AMER_CALL; }

static double intrinsic(const ref_option* o, double S) {
  double h = is_call(o->payoff) ? S - o->K : o->K - S;
  return h > 0.0 ? h : 0.0;
}

/* ------------------------------------------------------------------------- */
/* A plain static split of an index range over pthreads.                     */
/* ------------------------------------------------------------------------- */

typedef void (*range_fn)(void* ctx, int64_t begin, int64_t end);
typedef struct { range_fn fn; void* ctx; int64_t begin, end; } range_job;

static void* range_thread(void* arg) {
  range_job* j = (range_job*)arg;
  j->fn(j->ctx, j->begin, j->end);
  return NULL;
}

static void parallel_range(int64_t n, int nthreads, range_fn fn, void* ctx) {
  if (nthreads < 1) nthreads = 1;
  if (nthreads > 256) nthreads = 256;
  if ((int64_t)nthreads > n) nthreads = (int)(n > 0 ? n : 1);
  if (nthreads == 1) { fn(ctx, 0, n); return; }
  pthread_t th[256];
  range_job jobs[256];
  for (int t = 0; t < nthreads; ++t) {
    jobs[t].fn = fn;
    jobs[t].ctx = ctx;
    jobs[t].begin = n * t / nthreads;
    jobs[t].end = n * (t + 1) / nthreads;
    pthread_create(&th[t], NULL, range_thread, &jobs[t]);
  }
  for (int t = 0; t < nthreads; ++t) pthread_join(th[t], NULL);
}

/* ------------------------------------------------------------------------- */
/* Terminal values.                                                           */
/* ------------------------------------------------------------------------- */

typedef struct {
  const ref_option* o;
  int64_t path0;
  double *xT, *vT, *pay;
} sim_ctx;

static void sim_range(void* vctx, int64_t b, int64_t e) {
  sim_ctx* c = (sim_ctx*)vctx;
  const ref_option* o = c->o;
  double dt = o->T / o->steps;
  double disc = exp(-o->r * o->T);
  for (int64_t i = b; i < e; ++i) {
    int64_t path = c->path0 + i;
    double x = 0.0, v = o->v0;
    for (int32_t n = 0; n < o->steps; ++n) {
      double z1, z2, u, u2;
      draws_of(o, path, n, &z1, &z2, &u, &u2);
      transition(o, dt, &x, &v, z1, z2, u, u2);
    }
    if (c->xT) c->xT[i] = x;
    if (c->vT) c->vT[i] = v;
    if (c->pay) c->pay[i] = disc * intrinsic(o, o->S0 * exp(x));
  }
}

int ref_simulate(const ref_option* o, int64_t path0, int64_t npaths, int nthreads,
                 double* xT, double* vT, double* disc_payoff) {
  if (!o || npaths < 0 || o->steps < 1) return -1;
  sim_ctx c = {o, path0, xT, vT, disc_payoff};
  parallel_range(npaths, nthreads, sim_range, &c);
  return 0;
}

/* Mean and standard error of a sample, summed in index order in extended precision. */
static void mean_se(const double* a, int64_t n, double* mean, double* se, double sums[2]) {
  long double s = 0.0L, s2 = 0.0L;
  for (int64_t i = 0; i < n; ++i) {
    s += (long double)a[i];
    s2 += (long double)a[i] * (long double)a[i];
  }
  long double m = s / (long double)n;
  long double var = (s2 - s * s / (long double)n) / (long double)(n - 1);
  if (var < 0.0L) var = 0.0L;
  *mean = (double)m;
  *se = (double)sqrtl(var / (long double)n);
  if (sums) {
    sums[0] = (double)s;
    sums[1] = (double)s2;
  }
}

int ref_price_european(const ref_option* o, int nthreads, double* price, double* std_err,
                       double sums[2]) {
  if (!o || o->paths < 2) return -1;
  double* pay = (double*)malloc(sizeof(double) * (size_t)o->paths);
  if (!pay) return -1;
  ref_simulate(o, 0, o->paths, nthreads, NULL, NULL, pay);
  mean_se(pay, o->paths, price, std_err, sums);
  free(pay);
  return 0;
}

/* ------------------------------------------------------------------------- */
/* Longstaff-Schwartz.                                                        */
/* ------------------------------------------------------------------------- */

int ref_chol6_solve(const double G[36], const double b[6], double beta[6]) {
  double A[6][6], L[6][6], rhs[6], z[6], w[6];
  int perm[6];
  double maxd = 0.0;
  for (int i = 0; i < 6; ++i) {
    for (int j = 0; j < 6; ++j) {
      A[i][j] = G[i * 6 + j];
      L[i][j] = 0.0;
    }
    rhs[i] = b[i];
    perm[i] = i;
    beta[i] = 0.0;
    if (G[i * 6 + i] > maxd) maxd = G[i * 6 + i];
  }
  double tol = 1e-12 * maxd;
  int rank = 0;
  for (int k = 0; k < 6; ++k) {
    /* pivot: the largest remaining diagonal of the Schur complement (lowest index on ties) */
    int piv = k;
    for (int i = k + 1; i < 6; ++i)
      if (A[i][i] > A[piv][piv]) piv = i;
    if (!(A[piv][piv] > tol)) break; /* the remaining columns are dropped */
    if (piv != k) {
      for (int j = 0; j < 6; ++j) { double t = A[k][j]; A[k][j] = A[piv][j]; A[piv][j] = t; }
      for (int i = 0; i < 6; ++i) { double t = A[i][k]; A[i][k] = A[i][piv]; A[i][piv] = t; }
      for (int j = 0; j < k; ++j) { double t = L[k][j]; L[k][j] = L[piv][j]; L[piv][j] = t; }
      { double t = rhs[k]; rhs[k] = rhs[piv]; rhs[piv] = t; }
      { int t = perm[k]; perm[k] = perm[piv]; perm[piv] = t; }
    }
    L[k][k] = sqrt(A[k][k]);
    for (int i = k + 1; i < 6; ++i) L[i][k] = A[i][k] / L[k][k];
    for (int i = k + 1; i < 6; ++i)
      for (int j = k + 1; j < 6; ++j) A[i][j] -= L[i][k] * L[j][k];
    ++rank;
  }
  for (int i = 0; i < rank; ++i) { /* L z = rhs */
    double s = rhs[i];
    for (int j = 0; j < i; ++j) s -= L[i][j] * z[j];
    z[i] = s / L[i][i];
  }
  for (int i = rank - 1; i >= 0; --i) { /* L^T w = z */
    double s = z[i];
    for (int j = i + 1; j < rank; ++j) s -= L[j][i] * w[j];
    w[i] = s / L[i][i];
  }
  for (int i = 0; i < rank; ++i) beta[perm[i]] = w[i];
  return rank;
}

/* Regression basis at one exercise date: (1, a, a^2, c, a c, c^2) with
 * a = S/K - 1 and c = v/theta - 1.  It spans the same space as
 * {1, S, S^2, v, S v, v^2}, so the least-squares projection is the same; the
 * shift and scale only keep the normal equations well conditioned. */
static void lsm_basis(const ref_option* o, double S, double v, double phi[6]) {
  double a = (S - o->K) / o->K;
  double c = ((v > 0.0 ? v : 0.0) - o->theta) / o->theta;
  phi[0] = 1.0;
  phi[1] = a;
  phi[2] = a * a;
  phi[3] = c;
  phi[4] = a * c;
  phi[5] = c * c;
}

typedef struct {
  const ref_option* o;
  double *X, *V; /* [(n-1) * P + p] for n = 1..N */
} spill_ctx;

static void spill_range(void* vctx, int64_t b, int64_t e) {
  spill_ctx* c = (spill_ctx*)vctx;
  const ref_option* o = c->o;
  int64_t P = o->paths;
  double dt = o->T / o->steps;
  for (int64_t p = b; p < e; ++p) {
    double x = 0.0, v = o->v0;
    for (int32_t n = 0; n < o->steps; ++n) {
      double z1, z2, u, u2;
      draws_of(o, p, n, &z1, &z2, &u, &u2);
      transition(o, dt, &x, &v, z1, z2, u, u2);
      c->X[(size_t)n * P + p] = x;
      c->V[(size_t)n * P + p] = v;
    }
  }
}

int ref_path_states(const ref_option* o, int nthreads, double* X, double* V) {
  if (!o || !X || !V || o->steps < 1) return -1;
  spill_ctx sc = {o, X, V};
  parallel_range(o->paths, nthreads, spill_range, &sc);
  return 0;
}

int ref_price_american(const ref_option* o, int nthreads, double* price, double* std_err,
                       int32_t* tau_out, int32_t* exercised_at_t0, int32_t* lsm_flags) {
  return ref_price_american_beta(o, nthreads, price, std_err, tau_out, exercised_at_t0, lsm_flags, NULL);
}

int ref_price_american_beta(const ref_option* o, int nthreads, double* price, double* std_err,
                            int32_t* tau_out, int32_t* exercised_at_t0, int32_t* lsm_flags, double* beta_out) {
  if (!o || o->paths < 2 || o->steps < 1) return -1;
  const int64_t P = o->paths;
  const int32_t N = o->steps;
  const double dt = o->T / N;
  const double df = exp(-o->r * dt);
  double* X = (double*)malloc(sizeof(double) * (size_t)P * N);
  double* V = (double*)malloc(sizeof(double) * (size_t)P * N);
  double* Y = (double*)malloc(sizeof(double) * (size_t)P);
  int32_t* tau = (int32_t*)malloc(sizeof(int32_t) * (size_t)P);
  if (!X || !V || !Y || !tau) {
    free(X); free(V); free(Y); free(tau);
    return -1;
  }
  /* forward: every path's state at every exercise date (the path write-out) */
  spill_ctx sc = {o, X, V};
  parallel_range(P, nthreads, spill_range, &sc);

  int32_t flags = 0;
  /* cash flow at maturity */
  for (int64_t p = 0; p < P; ++p) {
    Y[p] = intrinsic(o, o->S0 * exp(X[(size_t)(N - 1) * P + p]));
    tau[p] = N;
  }
  /* backward induction over t_{N-1} .. t_1 */
  for (int32_t n = N - 1; n >= 1; --n) {
    const double* Xn = X + (size_t)(n - 1) * P;
    const double* Vn = V + (size_t)(n - 1) * P;
    long double G[36] = {0}, bsum[6] = {0};
    int64_t itm = 0;
    for (int64_t p = 0; p < P; ++p) {
      Y[p] *= df; /* the cash flow, discounted to t_n */
      double S = o->S0 * exp(Xn[p]);
      if (intrinsic(o, S) > 0.0) {
        double phi[6];
        lsm_basis(o, S, Vn[p], phi);
        for (int i = 0; i < 6; ++i) {
          for (int j = 0; j < 6; ++j) G[i * 6 + j] += (long double)(phi[i] * phi[j]);
          bsum[i] += (long double)(phi[i] * Y[p]);
        }
        ++itm;
      }
    }
    if (itm < 6) {
      flags |= 1;
      continue;
    }
    double Gd[36], bd[6], beta[6];
    for (int i = 0; i < 36; ++i) Gd[i] = (double)G[i];
    for (int i = 0; i < 6; ++i) bd[i] = (double)bsum[i];
    if (ref_chol6_solve(Gd, bd, beta) < 6) flags |= 2;
    if (beta_out)
      for (int i = 0; i < 6; ++i) beta_out[(size_t)n * 6 + i] = beta[i];
    for (int64_t p = 0; p < P; ++p) {
      double S = o->S0 * exp(Xn[p]);
      double h = intrinsic(o, S);
      if (h > 0.0) {
        double phi[6];
        lsm_basis(o, S, Vn[p], phi);
        double cont = 0.0;
        for (int i = 0; i < 6; ++i) cont += phi[i] * beta[i];
        if (h > cont) {
          Y[p] = h;
          tau[p] = n;
        }
      }
    }
  }
  double meanY, seY;
  mean_se(Y, P, &meanY, &seY, NULL);
  double cont0 = df * meanY;
  double h0 = intrinsic(o, o->S0);
  int ex0 = h0 > cont0;
  *price = ex0 ? h0 : cont0;
  *std_err = ex0 ? 0.0 : df * seY;
  if (exercised_at_t0) *exercised_at_t0 = ex0;
  if (lsm_flags) *lsm_flags = flags;
  if (tau_out) memcpy(tau_out, tau, sizeof(int32_t) * (size_t)P);
  free(X); free(V); free(Y); free(tau);
  return 0;
}

/* ------------------------------------------------------------------------- */
/* Stopped cash flows with given exercise indices (for checks of the Greeks). */
/* ------------------------------------------------------------------------- */

typedef struct {
  const ref_option* o;
  const int32_t* tau;
  double* out;
} stop_ctx;

static void stop_range(void* vctx, int64_t b, int64_t e) {
  stop_ctx* c = (stop_ctx*)vctx;
  const ref_option* o = c->o;
  double dt = o->T / o->steps;
  for (int64_t p = b; p < e; ++p) {
    double x = 0.0, v = o->v0;
    for (int32_t n = 0; n < c->tau[p]; ++n) {
      double z1, z2, u, u2;
      draws_of(o, p, n, &z1, &z2, &u, &u2);
      transition(o, dt, &x, &v, z1, z2, u, u2);
    }
    c->out[p] = exp(-o->r * (dt * c->tau[p])) * intrinsic(o, o->S0 * exp(x));
  }
}

int ref_stopped_values(const ref_option* o, const int32_t* tau, int nthreads, double* out) {
  if (!o || !tau || !out) return -1;
  for (int64_t p = 0; p < o->paths; ++p)
    if (tau[p] < 0 || tau[p] > o->steps) return -1;
  stop_ctx c = {o, tau, out};
  parallel_range(o->paths, nthreads, stop_range, &c);
  return 0;
}

/* ------------------------------------------------------------------------- */
/* Forward-mode pathwise Greeks.                                              */
/* ------------------------------------------------------------------------- */

/* Parameter order of the 7 tangent directions. */
/* tangent directions: the 7 model/contract parameters and the maturity T */
enum { D_S0 = 0, D_V0 = 1, D_THETA = 2, D_R = 3, D_KAPPA = 4, D_XI = 5, D_RHO = 6, D_T = 7, ND = 8 };

typedef struct { double v, d[ND]; } tanv;

static tanv tconst(double a) { tanv t; t.v = a; for (int i = 0; i < ND; ++i) t.d[i] = 0.0; return t; }
static tanv tseed(double a, int i) { tanv t = tconst(a); t.d[i] = 1.0; return t; }
static tanv tadd(tanv a, tanv b) { tanv t; t.v = a.v + b.v; for (int i = 0; i < ND; ++i) t.d[i] = a.d[i] + b.d[i]; return t; }
static tanv tsub(tanv a, tanv b) { tanv t; t.v = a.v - b.v; for (int i = 0; i < ND; ++i) t.d[i] = a.d[i] - b.d[i]; return t; }
static tanv tmul(tanv a, tanv b) { tanv t; t.v = a.v * b.v; for (int i = 0; i < ND; ++i) t.d[i] = a.d[i] * b.v + a.v * b.d[i]; return t; }
static tanv tdiv(tanv a, tanv b) {
  tanv t;
  t.v = a.v / b.v;
  for (int i = 0; i < ND; ++i) t.d[i] = (a.d[i] - t.v * b.d[i]) / b.v;
  return t;
}
static tanv tsqrt(tanv a) { /* the derivative at 0 is taken as 0 */
  tanv t;
  t.v = sqrt(a.v);
  for (int i = 0; i < ND; ++i) t.d[i] = (t.v > 0.0) ? a.d[i] / (2.0 * t.v) : 0.0;
  return t;
}
static tanv tlog(tanv a) { tanv t; t.v = log(a.v); for (int i = 0; i < ND; ++i) t.d[i] = a.d[i] / a.v; return t; }
static tanv texp(tanv a) { tanv t; t.v = exp(a.v); for (int i = 0; i < ND; ++i) t.d[i] = a.d[i] * t.v; return t; }
static tanv tscale(tanv a, double s) { tanv t; t.v = a.v * s; for (int i = 0; i < ND; ++i) t.d[i] = a.d[i] * s; return t; }

typedef struct {
  tanv S0, v0, theta, r, kappa, xi, rho, T, dtt; /* dtt = T / N */
  tanv E, omE, A1, A2, K[5], rdt, sqrt1mr2;
  double dt;
} tparams;

/* Model constants as functions of the 7 parameters, in the same operation
 * order as the plain steps above (so the primal parts agree bit for bit). */
static void tparams_init(const ref_option* o, tparams* tp) {
  double dt = o->T / o->steps;
  tp->dt = dt;
  tp->S0 = tseed(o->S0, D_S0);
  tp->v0 = tseed(o->v0, D_V0);
  tp->theta = tseed(o->theta, D_THETA);
  tp->r = tseed(o->r, D_R);
  tp->kappa = tseed(o->kappa, D_KAPPA);
  tp->xi = tseed(o->xi, D_XI);
  tp->rho = tseed(o->rho, D_RHO);
  tp->T = tseed(o->T, D_T);
  tp->dtt = tscale(tp->T, 1.0 / o->steps);
  tp->dtt.v = dt; /* the primal is T / N itself; its tangent is e_T / N */
  tanv mdt = tscale(tp->dtt, -1.0);
  tp->E = texp(tmul(tp->kappa, mdt));
  tp->omE = tsub(tconst(1.0), tp->E);
  tanv xi2 = tmul(tp->xi, tp->xi);
  tp->A1 = tdiv(tmul(tmul(xi2, tp->E), tp->omE), tp->kappa);
  tp->A2 = tdiv(tmul(tmul(tp->theta, xi2), tmul(tp->omE, tp->omE)), tscale(tp->kappa, 2.0));
  tp->rdt = tmul(tp->r, tp->dtt);
  /* gamma1 dt and gamma2 dt: products with 1/2, exact, so the primals equal the pricing run's */
  tanv g1dt = tscale(tp->dtt, GAMMA1), g2dt = tscale(tp->dtt, GAMMA2);
  if (o->xi > 0.0) {
    tanv rox = tdiv(tp->rho, tp->xi);
    tp->K[0] = tdiv(tmul(tmul(tmul(tp->rho, tp->kappa), tp->theta), mdt), tp->xi);
    /* K0 = -((rho kappa) theta dt)/xi: negation commutes exactly with the products */
    tanv core = tsub(tmul(tp->kappa, rox), tconst(0.5));
    tp->K[1] = tsub(tmul(core, g1dt), rox);
    tp->K[2] = tadd(tmul(core, g2dt), rox);
    tanv omr2 = tsub(tconst(1.0), tmul(tp->rho, tp->rho));
    tp->K[3] = tmul(omr2, g1dt);
    tp->K[4] = tmul(omr2, g2dt);
  } else {
    tp->K[0] = tconst(0.0);
    tp->K[1] = tscale(g1dt, 0.0 - 0.5);
    tp->K[2] = tscale(g2dt, 0.0 - 0.5);
    tp->K[3] = g1dt;
    tp->K[4] = g2dt;
  }
  tp->sqrt1mr2 = tsqrt(tsub(tconst(1.0), tmul(tp->rho, tp->rho)));
}

static tanv qe_variance_tan(const tparams* tp, tanv v, double z1, double u) {
  tanv m = tadd(tp->theta, tmul(tsub(v, tp->theta), tp->E));
  tanv s2 = tadd(tmul(v, tp->A1), tp->A2);
  if (!(s2.v > 0.0)) return m;
  tanv psi = tdiv(s2, tmul(m, m));
  if (psi.v <= PSI_C) {
    tanv t = tdiv(tconst(2.0), psi);
    tanv tm1 = tsub(t, tconst(1.0));
    tanv b2 = tadd(tm1, tmul(tsqrt(t), tsqrt(tm1)));
    tanv b = tsqrt(b2);
    tanv a = tdiv(m, tadd(tconst(1.0), b2));
    tanv bz = tadd(b, tconst(z1));
    return tmul(a, tmul(bz, bz));
  }
  tanv p = tdiv(tsub(psi, tconst(1.0)), tadd(psi, tconst(1.0)));
  tanv omp = tsub(tconst(1.0), p);
  tanv beta = tdiv(omp, m);
  if (u <= p.v) return tconst(0.0);
  return tdiv(tlog(tdiv(omp, tconst(1.0 - u))), beta);
}

/* The truncated Gaussian variance step in tangent arithmetic: V = max(r sigma + sigma Z1, 0) with
 * sigma = m / A(r), A(r) = r Phi(r) + phi(r), and r = r(psi) the root of B(r) / A(r)^2 = 1 + psi,
 * B(r) = (r^2 + 1) Phi(r) + r phi(r).  Since A' = Phi and B' = 2 A, the ratio's derivative is
 * 2 (A^2 - B Phi) / A^3, so dr/dpsi = A^3 / (2 (A^2 - B Phi)) by implicit differentiation.
 * The primal takes the operations of ref_tg_variance_step in its order. */
static tanv tg_variance_tan(const tparams* tp, tanv v, double z1) {
  tanv m = tadd(tp->theta, tmul(tsub(v, tp->theta), tp->E));
  tanv s2 = tadd(tmul(v, tp->A1), tp->A2);
  if (!(s2.v > 0.0)) return m;
  tanv psi = tdiv(s2, tmul(m, m));
  double r = ref_tg_r(psi.v);
  double P = std_cdf(r), f = std_pdf(r);
  double A = r * P + f, B = (r * r + 1.0) * P + r * f;
  double drdpsi = A * A * A / (2.0 * (A * A - B * P));
  tanv rt = tscale(psi, drdpsi);
  rt.v = r;
  tanv At = tscale(rt, P); /* dA = Phi dr */
  At.v = A;
  tanv sigma = tdiv(m, At);
  tanv V = tadd(tmul(rt, sigma), tscale(sigma, z1));
  return V.v > 0.0 ? V : tconst(0.0);
}

/* ln E[exp(A V_{n+1}) | v] in tangent arithmetic: the branch formulas of ref_qe_log_mgf on the
 * pricing run's primals (same moments, branch choice and existence test). */
static tanv qe_log_mgf_tan(const tparams* tp, tanv v, tanv A, int* ok) {
  tanv m = tadd(tp->theta, tmul(tsub(v, tp->theta), tp->E));
  tanv s2 = tadd(tmul(v, tp->A1), tp->A2);
  *ok = 1;
  if (!(s2.v > 0.0)) return tmul(A, m);
  tanv psi = tdiv(s2, tmul(m, m));
  if (psi.v <= PSI_C) {
    tanv t = tdiv(tconst(2.0), psi);
    tanv tm1 = tsub(t, tconst(1.0));
    tanv b2 = tadd(tm1, tmul(tsqrt(t), tsqrt(tm1)));
    tanv a = tdiv(m, tadd(tconst(1.0), b2));
    tanv d = tsub(tconst(1.0), tmul(tscale(A, 2.0), a));
    if (!(d.v > 0.0)) { *ok = 0; return tconst(0.0); }
    return tsub(tdiv(tmul(tmul(A, b2), a), d), tscale(tlog(d), 0.5));
  }
  tanv p = tdiv(tsub(psi, tconst(1.0)), tadd(psi, tconst(1.0)));
  tanv beta = tdiv(tsub(tconst(1.0), p), m);
  if (!(A.v < beta.v)) { *ok = 0; return tconst(0.0); }
  return tlog(tadd(p, tdiv(tmul(beta, tsub(tconst(1.0), p)), tsub(beta, A))));
}

/* One transition in tangent arithmetic; returns the coefficient of z2 in the log-price
 * increment (the conditional standard deviation of its Gaussian part). */
static double transition_tan(const ref_option* o, const tparams* tp, tanv* x, tanv* v,
                             double z1, double z2, double u) {
  if (o->scheme == REF_SCHEME_FTE) {
    tanv vp = (v->v > 0.0) ? *v : tconst(0.0);
    tanv sq = tsqrt(tmul(vp, tp->dtt));
    tanv zs = tadd(tscale(tp->rho, z1), tscale(tp->sqrt1mr2, z2));
    tanv vn = tadd(tadd(*v, tmul(tmul(tp->kappa, tsub(tp->theta, vp)), tp->dtt)),
                   tscale(tmul(tp->xi, sq), z1));
    *x = tadd(tadd(*x, tmul(tsub(tp->r, tscale(vp, 0.5)), tp->dtt)), tmul(sq, zs));
    *v = vn;
    return sq.v * tp->sqrt1mr2.v;
  }
  tanv vn = (o->scheme == REF_SCHEME_TG) ? tg_variance_tan(tp, *v, z1) : qe_variance_tan(tp, *v, z1, u);
  tanv w = tadd(tmul(tp->K[3], *v), tmul(tp->K[4], vn));
  tanv xn = tadd(*x, tp->rdt);
  if (o->scheme == REF_SCHEME_QE_M) {
    /* K0* = -ln E[exp(A V)] - (K1 + K3 / 2) v, A = K2 + K4 / 2, where the moment exists */
    tanv A = tadd(tp->K[2], tscale(tp->K[4], 0.5));
    int ok;
    tanv lm = qe_log_mgf_tan(tp, *v, A, &ok);
    tanv k0 = ok ? tsub(tscale(lm, -1.0), tmul(tadd(tp->K[1], tscale(tp->K[3], 0.5)), *v)) : tp->K[0];
    xn = tadd(xn, k0);
  } else {
    xn = tadd(xn, tp->K[0]);
  }
  xn = tadd(xn, tmul(tp->K[1], *v));
  xn = tadd(xn, tmul(tp->K[2], vn));
  tanv sw = tsqrt(w);
  xn = tadd(xn, tscale(sw, z2));
  *x = xn;
  *v = vn;
  return sw.v;
}

typedef struct {
  const ref_option* o;
  const tparams* tp;
  const int32_t* tau;   /* NULL for European */
  double* val;          /* [P] discounted cash flow */
  double* der;          /* [P * NG]: its 8 tangents, then the gamma term */
} greek_ctx;

enum { NG = ND + 1 }; /* Greeks per path: the 8 tangent directions and gamma */

static void greek_range(void* vctx, int64_t b, int64_t e) {
  greek_ctx* c = (greek_ctx*)vctx;
  const ref_option* o = c->o;
  const tparams* tp = c->tp;
  for (int64_t p = b; p < e; ++p) {
    int32_t stop = c->tau ? c->tau[p] : o->steps;
    tanv x = tconst(0.0), v = tp->v0;
    /* gamma: conditional on the variance path, x_stop is Gaussian in the asset variates z2 with
     * sum sigma_n^2 variance; the likelihood ratio of a shift of ln S0 is
     * W = sum sigma_n z2_n / sum sigma_n^2, so d2V/d(ln S0)^2 = E[xbar W] (xbar the pathwise
     * derivative of X in ln S0) and gamma = E[xbar (W - 1)] / S0^2 */
    double sz = 0.0, ss = 0.0;
    for (int32_t n = 0; n < stop; ++n) {
      double z1, z2, u, u2;
      draws_of(o, p, n, &z1, &z2, &u, &u2);
      double sig = transition_tan(o, tp, &x, &v, z1, z2, u);
      sz += sig * z2;
      ss += sig * sig;
    }
    tanv S = tmul(tp->S0, texp(x));
    tanv h = is_call(o->payoff) ? tsub(S, tconst(o->K)) : tsub(tconst(o->K), S);
    if (!(h.v > 0.0)) h = tconst(0.0);
    tanv disc = texp(tmul(tp->r, tscale(tp->dtt, -(double)stop)));
    if (!c->tau) disc = texp(tmul(tp->r, tscale(tp->T, -1.0)));
    tanv X = tmul(disc, h);
    c->val[p] = X.v;
    for (int i = 0; i < ND; ++i) c->der[(size_t)p * NG + i] = X.d[i];
    /* European only: with exercise indices decided on the same paths, re-weighting the paths
     * would carry each path's stopping decision onto trajectories it was not decided on, so
     * there is no gamma of this kind for a stopping rule (NaN) */
    double gam = 0.0; /* stopped at t_0 (no step): h(S0) is linear in S0 */
    if (c->tau) gam = NAN;
    else if (X.d[D_S0] != 0.0 && stop > 0) gam = (ss > 0.0) ? X.d[D_S0] * (sz / ss - 1.0) / o->S0 : NAN;
    c->der[(size_t)p * NG + ND] = gam;
  }
}

/* Mean and standard error of the discounted cash flow and of its 7 tangents, every path
 * stopped at tau[p] (at T when tau is NULL). */
static int greeks_at(const ref_option* o, const int32_t* tau, int nthreads, double* price, double* std_err,
                     double* grads, double* grad_se, int nout) {
  const int64_t P = o->paths;
  tparams tp;
  tparams_init(o, &tp);
  double* val = (double*)malloc(sizeof(double) * (size_t)P);
  double* der = (double*)malloc(sizeof(double) * (size_t)P * NG);
  double* col = (double*)malloc(sizeof(double) * (size_t)P);
  if (!val || !der || !col) {
    free(val); free(der); free(col);
    return -1;
  }
  greek_ctx gc = {o, &tp, tau, val, der};
  parallel_range(P, nthreads, greek_range, &gc);
  mean_se(val, P, price, std_err, NULL);
  for (int i = 0; i < nout; ++i) {
    for (int64_t p = 0; p < P; ++p) col[p] = der[(size_t)p * NG + i];
    mean_se(col, P, &grads[i], &grad_se[i], NULL);
  }
  free(val); free(der); free(col);
  return 0;
}

static int greeks_impl(const ref_option* o, int nthreads, double* price, double* std_err, double* grads,
                       double* grad_se, int nout) {
  if (!o || o->paths < 2 || o->steps < 1 || o->scheme == REF_SCHEME_BK) return -1;
  const int64_t P = o->paths;
  int american = (o->payoff == REF_AMER_PUT || o->payoff == REF_AMER_CALL);
  if (!american) return greeks_at(o, NULL, nthreads, price, std_err, grads, grad_se, nout);
  int32_t* tau = (int32_t*)malloc(sizeof(int32_t) * (size_t)P);
  if (!tau) return -1;
  int32_t ex0 = 0;
  double amer_price = 0.0, amer_se = 0.0, m, se;
  int rc = ref_price_american(o, nthreads, &amer_price, &amer_se, tau, &ex0, NULL);
  if (rc == 0 && ex0) { /* exercised at t_0: the value is the intrinsic h(S0), linear in S0 */
    for (int i = 0; i < nout; ++i) { grads[i] = 0.0; grad_se[i] = 0.0; }
    grads[D_S0] = is_call(o->payoff) ? 1.0 : -1.0;
    amer_se = 0.0;
  } else if (rc == 0) {
    rc = greeks_at(o, tau, nthreads, &m, &se, grads, grad_se, nout);
  }
  free(tau);
  if (rc) return rc;
  *price = amer_price;
  *std_err = amer_se;
  return 0;
}

int ref_greeks(const ref_option* o, int nthreads, double* price, double* std_err,
               double grads[7], double grad_se[7]) {
  return greeks_impl(o, nthreads, price, std_err, grads, grad_se, 7);
}

int ref_greeks_ext(const ref_option* o, int nthreads, double* price, double* std_err,
                   double grads[9], double grad_se[9]) {
  return greeks_impl(o, nthreads, price, std_err, grads, grad_se, NG);
}

static int greeks_at_tau_impl(const ref_option* o, const int32_t* tau, int nthreads, double* value,
                              double* std_err, double* grads, double* grad_se, int nout) {
  if (!o || !tau || o->paths < 2 || o->steps < 1 || o->scheme == REF_SCHEME_BK) return -1;
  for (int64_t p = 0; p < o->paths; ++p)
    if (tau[p] < 0 || tau[p] > o->steps) return -1;
  return greeks_at(o, tau, nthreads, value, std_err, grads, grad_se, nout);
}

int ref_greeks_at_tau(const ref_option* o, const int32_t* tau, int nthreads, double* value, double* std_err,
                      double grads[7], double grad_se[7]) {
  return greeks_at_tau_impl(o, tau, nthreads, value, std_err, grads, grad_se, 7);
}

int ref_greeks_at_tau_ext(const ref_option* o, const int32_t* tau, int nthreads, double* value, double* std_err,
                          double grads[9], double grad_se[9]) {
  return greeks_at_tau_impl(o, tau, nthreads, value, std_err, grads, grad_se, NG);
}

/* ------------------------------------------------------------------------- */
/* Correlated baskets (the paper's asset dimension as correlated underlyings). */
/* ------------------------------------------------------------------------- */

#define LDC REF_MAX_ASSETS

int ref_corr_cholesky(int d, const double* C, double* L) {
  if (d < 1 || d > REF_MAX_ASSETS) return -1;
  for (int i = 0; i < d; ++i)
    for (int j = 0; j < d; ++j) L[i * LDC + j] = 0.0;
  /* Cholesky-Banachiewicz, row by row: L_ij = (C_ij - sum_k<j L_ik L_jk) / L_jj */
  for (int i = 0; i < d; ++i) {
    for (int j = 0; j <= i; ++j) {
      double s = C[i * LDC + j];
      for (int k = 0; k < j; ++k) s -= L[i * LDC + k] * L[j * LDC + k];
      if (i == j) {
        if (!(s > 0.0)) return -1;
        L[i * LDC + i] = sqrt(s);
      } else {
        L[i * LDC + j] = s / L[j * LDC + j];
      }
    }
  }
  return 0;
}

/* Asset i of the basket seen as a single-asset option (its own Heston parameters). */
static void asset_view(const ref_basket* b, int i, ref_option* o) {
  memset(o, 0, sizeof *o);
  o->S0 = b->S0[i];
  o->K = b->K;
  o->T = b->T;
  o->r = b->r;
  o->kappa = b->kappa[i];
  o->theta = b->theta[i];
  o->xi = b->xi[i];
  o->rho = b->rho[i];
  o->v0 = b->v0[i];
  o->payoff = REF_EURO_CALL;
  o->steps = b->steps;
  o->paths = b->paths;
  o->seed = b->seed;
  o->stream = b->stream;
  o->scheme = b->scheme;
}

/* Coefficient of the (correlated) asset normal in one log-price increment. */
static double z2_coeff(const ref_option* o, double dt, double v, double vn) {
  if (o->scheme == REF_SCHEME_FTE) {
    double vp = v > 0.0 ? v : 0.0;
    return sqrt(vp * dt) * sqrt(1.0 - o->rho * o->rho);
  }
  double K[5];
  qe_k_coeffs(o->kappa, o->theta, o->xi, o->rho, dt, K);
  return sqrt(K[3] * v + K[4] * vn);
}

typedef struct {
  const ref_basket* b;
  ref_option view[REF_MAX_ASSETS];
  double L[REF_MAX_ASSETS * REF_MAX_ASSETS];
  double dt;
} basket_setup;

static int basket_setup_init(const ref_basket* b, basket_setup* s) {
  if (!b || b->assets < 1 || b->assets > REF_MAX_ASSETS || b->steps < 1 || b->scheme == REF_SCHEME_BK) return -1;
  s->b = b;
  for (int i = 0; i < b->assets; ++i) asset_view(b, i, &s->view[i]);
  s->dt = b->T / b->steps;
  return ref_corr_cholesky(b->assets, b->corr, s->L);
}

/* One transition n of all assets of a path.  Asset i draws its own words from the counter
 * (n, path, stream, i): Box-Muller (z1_i, z2_i) and the uniform u_i.  The asset normals are
 * correlated, zc = L z2, and asset i takes its own scheme's step with (z1_i, zc_i, u_i).
 * s[i] (may be NULL) receives the coefficient of zc_i in asset i's log-price increment and
 * zind (may be NULL) the independent normals z2. */
/* The draws of transition n of a path: asset i takes the words of counter (n, path, stream, i),
 * Box-Muller (z1_i, z2_i) and the uniform u_i. */
static void basket_draws(const ref_basket* b, int64_t path, int32_t n, double* z1, double* z2, double* u) {
  uint32_t key[2] = {(uint32_t)(b->seed & 0xffffffffu), (uint32_t)(b->seed >> 32)};
  for (int i = 0; i < b->assets; ++i) {
    uint32_t ctr[4] = {(uint32_t)n, (uint32_t)path, b->stream, (uint32_t)i};
    uint32_t w[4];
    ref_philox4x32_10(ctr, key, w);
    ref_box_muller(ref_uniform(w[0]), ref_uniform(w[1]), &z1[i], &z2[i]);
    u[i] = ref_uniform(w[2]);
  }
}

static void basket_transition(const basket_setup* S, int64_t path, int32_t n, double* x, double* v, double* s,
                              double* zind) {
  const ref_basket* b = S->b;
  const int d = b->assets;
  double z1[REF_MAX_ASSETS], z2[REF_MAX_ASSETS], u[REF_MAX_ASSETS];
  basket_draws(b, path, n, z1, z2, u);
  for (int i = 0; i < d; ++i) {
    double zc = 0.0;
    for (int k = 0; k <= i; ++k) zc += S->L[i * LDC + k] * z2[k];
    double vb = v[i];
    transition(&S->view[i], S->dt, &x[i], &v[i], z1[i], zc, u[i], 0.5);
    if (s) s[i] = z2_coeff(&S->view[i], S->dt, vb, v[i]);
    if (zind) zind[i] = z2[i];
  }
}

static void basket_init_state(const ref_basket* b, double* x, double* v) {
  for (int i = 0; i < b->assets; ++i) {
    x[i] = 0.0;
    v[i] = b->v0[i];
  }
}

static double basket_value(const ref_basket* b, const double* x) {
  double B = 0.0;
  for (int i = 0; i < b->assets; ++i) B += b->w[i] * (b->S0[i] * exp(x[i]));
  return B;
}

static double basket_b0(const ref_basket* b) {
  double B = 0.0;
  for (int i = 0; i < b->assets; ++i) B += b->w[i] * b->S0[i];
  return B;
}

static double basket_intrinsic(const ref_basket* b, double B) {
  double h = is_call(b->payoff) ? B - b->K : b->K - B;
  return h > 0.0 ? h : 0.0;
}

typedef struct {
  const basket_setup* S;
  int64_t path0;
  double *xT, *vT, *pay;
} bsim_ctx;

static void bsim_range(void* vctx, int64_t bgn, int64_t end) {
  bsim_ctx* c = (bsim_ctx*)vctx;
  const ref_basket* b = c->S->b;
  const int d = b->assets;
  double disc = exp(-b->r * b->T);
  for (int64_t i = bgn; i < end; ++i) {
    int64_t path = c->path0 + i;
    double x[REF_MAX_ASSETS], v[REF_MAX_ASSETS];
    basket_init_state(b, x, v);
    for (int32_t n = 0; n < b->steps; ++n) basket_transition(c->S, path, n, x, v, NULL, NULL);
    for (int k = 0; k < d; ++k) {
      if (c->xT) c->xT[i * d + k] = x[k];
      if (c->vT) c->vT[i * d + k] = v[k];
    }
    if (c->pay) c->pay[i] = disc * basket_intrinsic(b, basket_value(b, x));
  }
}

int ref_basket_simulate(const ref_basket* b, int64_t path0, int64_t npaths, int nthreads, double* xT, double* vT,
                        double* disc_payoff) {
  basket_setup S;
  if (npaths < 0 || basket_setup_init(b, &S)) return -1;
  bsim_ctx c = {&S, path0, xT, vT, disc_payoff};
  parallel_range(npaths, nthreads, bsim_range, &c);
  return 0;
}

int ref_basket_price_european(const ref_basket* b, int nthreads, double* price, double* std_err) {
  if (!b || b->paths < 2) return -1;
  double* pay = (double*)malloc(sizeof(double) * (size_t)b->paths);
  if (!pay) return -1;
  int rc = ref_basket_simulate(b, 0, b->paths, nthreads, NULL, NULL, pay);
  if (rc == 0) mean_se(pay, b->paths, price, std_err, NULL);
  free(pay);
  return rc;
}

/* Basket log-value and value-weighted variance at every date (the LSM write-out). */
typedef struct {
  const basket_setup* S;
  double *X, *V;
} bstate_ctx;

static void bstate_range(void* vctx, int64_t bgn, int64_t end) {
  bstate_ctx* c = (bstate_ctx*)vctx;
  const ref_basket* b = c->S->b;
  const int64_t P = b->paths;
  const double B0 = basket_b0(b);
  for (int64_t p = bgn; p < end; ++p) {
    double x[REF_MAX_ASSETS], v[REF_MAX_ASSETS];
    basket_init_state(b, x, v);
    for (int32_t n = 0; n < b->steps; ++n) {
      basket_transition(c->S, p, n, x, v, NULL, NULL);
      double B = 0.0, Bv = 0.0;
      for (int i = 0; i < b->assets; ++i) {
        double Si = b->w[i] * (b->S0[i] * exp(x[i]));
        B += Si;
        Bv += Si * (v[i] > 0.0 ? v[i] : 0.0);
      }
      c->X[(size_t)n * P + p] = log(B / B0);
      c->V[(size_t)n * P + p] = Bv / B;
    }
  }
}

int ref_basket_states(const ref_basket* b, int nthreads, double* X, double* V) {
  basket_setup S;
  if (!X || !V || basket_setup_init(b, &S)) return -1;
  bstate_ctx c = {&S, X, V};
  parallel_range(b->paths, nthreads, bstate_range, &c);
  return 0;
}

int ref_chol_solve(int nb, const double* G, const double* bv, double* beta) {
  enum { MX = 16 };
  if (nb < 1 || nb > MX) return -1;
  double A[MX][MX], L[MX][MX], rhs[MX], z[MX], w[MX];
  int perm[MX];
  double maxd = 0.0;
  for (int i = 0; i < nb; ++i) {
    for (int j = 0; j < nb; ++j) {
      A[i][j] = G[i * nb + j];
      L[i][j] = 0.0;
    }
    rhs[i] = bv[i];
    perm[i] = i;
    beta[i] = 0.0;
    if (G[i * nb + i] > maxd) maxd = G[i * nb + i];
  }
  double tol = 1e-12 * maxd;
  int rank = 0;
  for (int k = 0; k < nb; ++k) {
    int piv = k; /* largest remaining Schur diagonal, lowest index on ties */
    for (int i = k + 1; i < nb; ++i)
      if (A[i][i] > A[piv][piv]) piv = i;
    if (!(A[piv][piv] > tol)) break;
    if (piv != k) {
      for (int j = 0; j < nb; ++j) { double t = A[k][j]; A[k][j] = A[piv][j]; A[piv][j] = t; }
      for (int i = 0; i < nb; ++i) { double t = A[i][k]; A[i][k] = A[i][piv]; A[i][piv] = t; }
      for (int j = 0; j < k; ++j) { double t = L[k][j]; L[k][j] = L[piv][j]; L[piv][j] = t; }
      { double t = rhs[k]; rhs[k] = rhs[piv]; rhs[piv] = t; }
      { int t = perm[k]; perm[k] = perm[piv]; perm[piv] = t; }
    }
    L[k][k] = sqrt(A[k][k]);
    for (int i = k + 1; i < nb; ++i) L[i][k] = A[i][k] / L[k][k];
    for (int i = k + 1; i < nb; ++i)
      for (int j = k + 1; j < nb; ++j) A[i][j] -= L[i][k] * L[j][k];
    ++rank;
  }
  for (int i = 0; i < rank; ++i) {
    double s = rhs[i];
    for (int j = 0; j < i; ++j) s -= L[i][j] * z[j];
    z[i] = s / L[i][i];
  }
  for (int i = rank - 1; i >= 0; --i) {
    double s = z[i];
    for (int j = i + 1; j < rank; ++j) s -= L[j][i] * w[j];
    w[i] = s / L[i][i];
  }
  for (int i = 0; i < rank; ++i) beta[perm[i]] = w[i];
  return rank;
}

/* Basket regression basis: the full cubic in a = B/K - 1 and c = vbar/thetabar - 1,
 * (1, a, a^2, c, a c, c^2, a^3, a^2 c, a c^2, c^3); thetabar = sum w_i S0_i theta_i / B0. */
static void basket_basis(double a, double c, double phi[REF_BASKET_NB]) {
  phi[0] = 1.0;
  phi[1] = a;
  phi[2] = a * a;
  phi[3] = c;
  phi[4] = a * c;
  phi[5] = c * c;
  phi[6] = a * a * a;
  phi[7] = a * a * c;
  phi[8] = a * c * c;
  phi[9] = c * c * c;
}

static double basket_theta_bar(const ref_basket* b) {
  double s = 0.0;
  for (int i = 0; i < b->assets; ++i) s += b->w[i] * b->S0[i] * b->theta[i];
  return s / basket_b0(b);
}

int ref_basket_price_american(const ref_basket* b, int nthreads, double* price, double* std_err, int32_t* tau_out,
                              int32_t* exercised_at_t0, int32_t* lsm_flags, double* beta_out) {
  enum { NB = REF_BASKET_NB };
  if (!b || b->paths < 2 || b->steps < 1) return -1;
  const int64_t P = b->paths;
  const int32_t N = b->steps;
  const double dt = b->T / N;
  const double df = exp(-b->r * dt);
  const double B0 = basket_b0(b), thb = basket_theta_bar(b);
  double* X = (double*)malloc(sizeof(double) * (size_t)P * N);
  double* V = (double*)malloc(sizeof(double) * (size_t)P * N);
  double* Y = (double*)malloc(sizeof(double) * (size_t)P);
  int32_t* tau = (int32_t*)malloc(sizeof(int32_t) * (size_t)P);
  int rc = (X && V && Y && tau) ? ref_basket_states(b, nthreads, X, V) : -1;
  if (rc) {
    free(X); free(V); free(Y); free(tau);
    return -1;
  }
  int32_t flags = 0;
  for (int64_t p = 0; p < P; ++p) {
    Y[p] = basket_intrinsic(b, B0 * exp(X[(size_t)(N - 1) * P + p]));
    tau[p] = N;
  }
  for (int32_t n = N - 1; n >= 1; --n) {
    const double* Xn = X + (size_t)(n - 1) * P;
    const double* Vn = V + (size_t)(n - 1) * P;
    long double G[NB * NB] = {0}, bs[NB] = {0};
    int64_t itm = 0;
    for (int64_t p = 0; p < P; ++p) {
      Y[p] *= df;
      double B = B0 * exp(Xn[p]);
      if (basket_intrinsic(b, B) > 0.0) {
        double phi[NB];
        basket_basis((B - b->K) / b->K, (Vn[p] - thb) / thb, phi);
        for (int i = 0; i < NB; ++i) {
          for (int j = 0; j < NB; ++j) G[i * NB + j] += (long double)(phi[i] * phi[j]);
          bs[i] += (long double)(phi[i] * Y[p]);
        }
        ++itm;
      }
    }
    if (itm < NB) {
      flags |= 1;
      continue;
    }
    double Gd[NB * NB], bd[NB], beta[NB];
    for (int i = 0; i < NB * NB; ++i) Gd[i] = (double)G[i];
    for (int i = 0; i < NB; ++i) bd[i] = (double)bs[i];
    if (ref_chol_solve(NB, Gd, bd, beta) < NB) flags |= 2;
    if (beta_out)
      for (int i = 0; i < NB; ++i) beta_out[(size_t)n * NB + i] = beta[i];
    for (int64_t p = 0; p < P; ++p) {
      double B = B0 * exp(Xn[p]);
      double h = basket_intrinsic(b, B);
      if (h > 0.0) {
        double phi[NB];
        basket_basis((B - b->K) / b->K, (Vn[p] - thb) / thb, phi);
        double cont = 0.0;
        for (int i = 0; i < NB; ++i) cont += phi[i] * beta[i];
        if (h > cont) {
          Y[p] = h;
          tau[p] = n;
        }
      }
    }
  }
  double meanY, seY;
  mean_se(Y, P, &meanY, &seY, NULL);
  double cont0 = df * meanY;
  double h0 = basket_intrinsic(b, B0);
  int ex0 = h0 > cont0;
  *price = ex0 ? h0 : cont0;
  *std_err = ex0 ? 0.0 : df * seY;
  if (exercised_at_t0) *exercised_at_t0 = ex0;
  if (lsm_flags) *lsm_flags = flags;
  if (tau_out) memcpy(tau_out, tau, sizeof(int32_t) * (size_t)P);
  free(X); free(V); free(Y); free(tau);
  return 0;
}

/* Per path: the discounted stopped cash flow, the pathwise delta samples
 * D_i = e^{-r tau dt} h'(B_tau) w_i S_tau,i / S0_i and (stopping at N only) the
 * likelihood-ratio scores of ln S0_j, score_j = sum_n s_nj u_nj / sum_n s_nj^2 with
 * u_n = L^{-T} z2_n (NaN where sum_n s_nj^2 = 0). */
typedef struct {
  const basket_setup* S;
  const int32_t* tau; /* NULL: stop at N */
  double *val, *D, *score;
} bgreek_ctx;

static void bgreek_range(void* vctx, int64_t bgn, int64_t end) {
  bgreek_ctx* c = (bgreek_ctx*)vctx;
  const basket_setup* S = c->S;
  const ref_basket* b = S->b;
  const int d = b->assets;
  for (int64_t p = bgn; p < end; ++p) {
    const int32_t tp = c->tau ? c->tau[p] : b->steps;
    double x[REF_MAX_ASSETS], v[REF_MAX_ASSETS], sa[REF_MAX_ASSETS] = {0}, sb[REF_MAX_ASSETS] = {0};
    basket_init_state(b, x, v);
    for (int32_t n = 0; n < tp; ++n) {
      double s[REF_MAX_ASSETS], z2[REF_MAX_ASSETS], u[REF_MAX_ASSETS];
      basket_transition(S, p, n, x, v, s, z2);
      if (c->score) {
        /* L^T u = z2 by back substitution */
        for (int j = d - 1; j >= 0; --j) {
          double t = z2[j];
          for (int k = j + 1; k < d; ++k) t -= S->L[k * LDC + j] * u[k];
          u[j] = t / S->L[j * LDC + j];
        }
        for (int j = 0; j < d; ++j) {
          sa[j] += s[j] * u[j];
          sb[j] += s[j] * s[j];
        }
      }
    }
    const double disc = exp(-b->r * (S->dt * tp));
    const double B = basket_value(b, x);
    const double h = basket_intrinsic(b, B);
    const double dh = h > 0.0 ? (is_call(b->payoff) ? 1.0 : -1.0) : 0.0;
    c->val[p] = disc * h;
    for (int i = 0; i < d; ++i) c->D[(size_t)p * d + i] = disc * dh * b->w[i] * (b->S0[i] * exp(x[i])) / b->S0[i];
    if (c->score)
      for (int j = 0; j < d; ++j) c->score[(size_t)p * d + j] = sb[j] > 0.0 ? sa[j] / sb[j] : NAN;
  }
}

int ref_basket_greeks(const ref_basket* b, const int32_t* tau_in, int nthreads, double* price, double* std_err,
                      double* delta, double* delta_se, double* gamma, double* gamma_se) {
  basket_setup S;
  if (!b || b->paths < 2 || basket_setup_init(b, &S)) return -1;
  const int d = b->assets;
  const int64_t P = b->paths;
  const int amer = b->payoff == REF_AMER_PUT || b->payoff == REF_AMER_CALL;
  int32_t* tau = NULL;
  int ex0 = 0;
  double lsm_price = 0.0, lsm_se = 0.0;
  if (tau_in) {
    for (int64_t p = 0; p < P; ++p)
      if (tau_in[p] < 0 || tau_in[p] > b->steps) return -1;
  } else if (amer) {
    tau = (int32_t*)malloc(sizeof(int32_t) * (size_t)P);
    if (!tau || ref_basket_price_american(b, nthreads, &lsm_price, &lsm_se, tau, &ex0, NULL, NULL)) {
      free(tau);
      return -1;
    }
    if (ex0)
      for (int64_t p = 0; p < P; ++p) tau[p] = 0;
  }
  const int32_t* tu = tau_in ? tau_in : tau;
  const int want_gamma = tu == NULL;
  double* val = (double*)malloc(sizeof(double) * (size_t)P);
  double* D = (double*)malloc(sizeof(double) * (size_t)P * d);
  double* sc = want_gamma ? (double*)malloc(sizeof(double) * (size_t)P * d) : NULL;
  double* tmp = (double*)malloc(sizeof(double) * (size_t)P);
  if (!val || !D || !tmp || (want_gamma && !sc)) {
    free(tau); free(val); free(D); free(sc); free(tmp);
    return -1;
  }
  bgreek_ctx c = {&S, tu, val, D, sc};
  parallel_range(P, nthreads, bgreek_range, &c);
  mean_se(val, P, price, std_err, NULL);
  if (amer && !tau_in) {
    *price = lsm_price;
    *std_err = lsm_se;
  }
  for (int i = 0; i < d; ++i) {
    for (int64_t p = 0; p < P; ++p) tmp[p] = D[(size_t)p * d + i];
    mean_se(tmp, P, &delta[i], &delta_se[i], NULL);
  }
  for (int i = 0; i < d; ++i)
    for (int j = 0; j < d; ++j) {
      if (!want_gamma) {
        gamma[i * d + j] = NAN;
        gamma_se[i * d + j] = NAN;
        continue;
      }
      /* symmetrised pathwise-LR sample:
       * (D_i score_j / S0_j + D_j score_i / S0_i) / 2 - [i = j] D_i / S0_i */
      for (int64_t p = 0; p < P; ++p) {
        const double* Dp = D + (size_t)p * d;
        const double* sp = sc + (size_t)p * d;
        int any = 0;
        for (int k = 0; k < d; ++k) any |= Dp[k] != 0.0;
        if (!any) {
          tmp[p] = 0.0;
          continue;
        }
        double g = 0.5 * (Dp[i] * sp[j] / b->S0[j] + Dp[j] * sp[i] / b->S0[i]);
        if (i == j) g -= Dp[i] / b->S0[i];
        tmp[p] = g;
      }
      mean_se(tmp, P, &gamma[i * d + j], &gamma_se[i * d + j], NULL);
    }
  free(tau); free(val); free(D); free(sc); free(tmp);
  return 0;
}

/* ------------------------------------------------------------------------- */
/* Basket risk Greeks: vegas per asset and correlation sensitivities.         */
/* ------------------------------------------------------------------------- */

/* The Cholesky factor L of C together with its derivative dL in the symmetric direction
 * E_ij + E_ji (i != j: C_ij and C_ji move together): the Cholesky-Banachiewicz recursion of
 * ref_corr_cholesky carried out on (value, derivative) pairs. */
static int corr_cholesky_tan(int d, const double* C, int pi, int pj, double* L, double* dL) {
  for (int i = 0; i < d; ++i)
    for (int j = 0; j < d; ++j) L[i * LDC + j] = dL[i * LDC + j] = 0.0;
  for (int i = 0; i < d; ++i) {
    for (int j = 0; j <= i; ++j) {
      double s = C[i * LDC + j];
      double ds = ((i == pi && j == pj) || (i == pj && j == pi)) ? 1.0 : 0.0;
      for (int k = 0; k < j; ++k) {
        s -= L[i * LDC + k] * L[j * LDC + k];
        ds -= dL[i * LDC + k] * L[j * LDC + k] + L[i * LDC + k] * dL[j * LDC + k];
      }
      if (i == j) {
        if (!(s > 0.0)) return -1;
        L[i * LDC + i] = sqrt(s);
        dL[i * LDC + i] = ds / (2.0 * L[i * LDC + i]);
      } else {
        L[i * LDC + j] = s / L[j * LDC + j];
        dL[i * LDC + j] = (ds - L[i * LDC + j] * dL[j * LDC + j]) / L[j * LDC + j];
      }
    }
  }
  return 0;
}

int ref_corr_cholesky_tan(int d, const double* C, int i, int j, double* L, double* dL) {
  if (d < 1 || d > REF_MAX_ASSETS || i < 0 || j < 0 || i >= d || j >= d || i == j) return -1;
  return corr_cholesky_tan(d, C, i, j, L, dL);
}

typedef struct {
  const basket_setup* S;
  const tparams* tp;     /* per asset: the tangent constants of its own parameters */
  const double* dL;      /* per pair q of (i > j): d L / d C_ij, LDC x LDC */
  const int32_t* tau;    /* NULL: stop at N */
  double *val, *vv, *vt, *dc;
} brisk_ctx;

/* Per path: the discounted stopped cash flow X = e^{-r tau dt} h(B_tau); the vega samples
 * dX/dv0_i and dX/dtheta_i = e^{-r tau dt} h'(B) w_i S_i dx_i, dx_i the tangent of asset i's
 * log-price in its own v0 or theta (an asset's Heston parameters move its own path only); and
 * the correlation samples dX/dC_ij = e^{-r tau dt} h'(B) sum_k w_k S_k dx_k/dC_ij with
 * dx_k/dC_ij = sum_n s_nk (dL z2_n)_k = sum_m dL_km Q_km, s_nk the coefficient of zc_k in asset
 * k's increment of step n and Q_km = sum_n s_nk z2_nm. */
static void brisk_range(void* vctx, int64_t bgn, int64_t end) {
  brisk_ctx* c = (brisk_ctx*)vctx;
  const basket_setup* S = c->S;
  const ref_basket* b = S->b;
  const int d = b->assets;
  const int npair = d * (d - 1) / 2;
  for (int64_t p = bgn; p < end; ++p) {
    const int32_t stop = c->tau ? c->tau[p] : b->steps;
    tanv x[REF_MAX_ASSETS], v[REF_MAX_ASSETS];
    double Q[REF_MAX_ASSETS * REF_MAX_ASSETS];
    for (int i = 0; i < d; ++i) {
      x[i] = tconst(0.0);
      v[i] = c->tp[i].v0;
      for (int m = 0; m < d; ++m) Q[i * LDC + m] = 0.0;
    }
    for (int32_t n = 0; n < stop; ++n) {
      double z1[REF_MAX_ASSETS], z2[REF_MAX_ASSETS], u[REF_MAX_ASSETS];
      basket_draws(b, p, n, z1, z2, u);
      for (int i = 0; i < d; ++i) {
        double zc = 0.0;
        for (int k = 0; k <= i; ++k) zc += S->L[i * LDC + k] * z2[k];
        const double sw = transition_tan(&S->view[i], &c->tp[i], &x[i], &v[i], z1[i], zc, u[i]);
        for (int m = 0; m <= i; ++m) Q[i * LDC + m] += sw * z2[m];
      }
    }
    double xv[REF_MAX_ASSETS];
    for (int i = 0; i < d; ++i) xv[i] = x[i].v;
    const double disc = exp(-b->r * (S->dt * stop));
    const double B = basket_value(b, xv);
    const double h = basket_intrinsic(b, B);
    const double dh = h > 0.0 ? (is_call(b->payoff) ? 1.0 : -1.0) : 0.0;
    c->val[p] = disc * h;
    double a[REF_MAX_ASSETS]; /* e^{-r tau dt} h'(B) w_k S_k */
    for (int k = 0; k < d; ++k) a[k] = disc * dh * b->w[k] * (b->S0[k] * exp(xv[k]));
    for (int i = 0; i < d; ++i) {
      c->vv[(size_t)p * d + i] = a[i] * x[i].d[D_V0];
      c->vt[(size_t)p * d + i] = a[i] * x[i].d[D_THETA];
    }
    for (int q = 0; q < npair; ++q) {
      const double* dLq = c->dL + (size_t)q * LDC * LDC;
      double g = 0.0;
      for (int k = 0; k < d; ++k) {
        double t = 0.0;
        for (int m = 0; m <= k; ++m) t += dLq[k * LDC + m] * Q[k * LDC + m];
        g += a[k] * t;
      }
      c->dc[(size_t)p * npair + q] = g;
    }
  }
}

int ref_basket_risk_greeks(const ref_basket* b, const int32_t* tau_in, int nthreads, double* price, double* std_err,
                           double* vega_v0, double* vega_v0_se, double* vega_theta, double* vega_theta_se,
                           double* dcorr, double* dcorr_se) {
  basket_setup S;
  if (!b || b->paths < 2 || basket_setup_init(b, &S)) return -1;
  const int d = b->assets;
  const int64_t P = b->paths;
  const int npair = d * (d - 1) / 2;
  const int amer = b->payoff == REF_AMER_PUT || b->payoff == REF_AMER_CALL;
  int32_t* tau = NULL;
  int ex0 = 0;
  double lsm_price = 0.0, lsm_se = 0.0;
  if (tau_in) {
    for (int64_t p = 0; p < P; ++p)
      if (tau_in[p] < 0 || tau_in[p] > b->steps) return -1;
  } else if (amer) {
    tau = (int32_t*)malloc(sizeof(int32_t) * (size_t)P);
    if (!tau || ref_basket_price_american(b, nthreads, &lsm_price, &lsm_se, tau, &ex0, NULL, NULL)) {
      free(tau);
      return -1;
    }
    if (ex0)
      for (int64_t p = 0; p < P; ++p) tau[p] = 0;
  }
  const int32_t* tu = tau_in ? tau_in : tau;
  tparams tp[REF_MAX_ASSETS];
  for (int i = 0; i < d; ++i) tparams_init(&S.view[i], &tp[i]);
  double* dL = (double*)malloc(sizeof(double) * (size_t)(npair > 0 ? npair : 1) * LDC * LDC);
  double* val = (double*)malloc(sizeof(double) * (size_t)P);
  double* vv = (double*)malloc(sizeof(double) * (size_t)P * d);
  double* vt = (double*)malloc(sizeof(double) * (size_t)P * d);
  double* dc = (double*)malloc(sizeof(double) * (size_t)P * (npair > 0 ? npair : 1));
  double* tmp = (double*)malloc(sizeof(double) * (size_t)P);
  int rc = (!dL || !val || !vv || !vt || !dc || !tmp) ? -1 : 0;
  double Lt[LDC * LDC];
  for (int i = 1; i < d && rc == 0; ++i)
    for (int j = 0; j < i && rc == 0; ++j)
      rc = corr_cholesky_tan(d, b->corr, i, j, Lt, dL + (size_t)(i * (i - 1) / 2 + j) * LDC * LDC);
  if (rc == 0) {
    brisk_ctx c = {&S, tp, dL, tu, val, vv, vt, dc};
    parallel_range(P, nthreads, brisk_range, &c);
    mean_se(val, P, price, std_err, NULL);
    if (amer && !tau_in) {
      *price = lsm_price;
      *std_err = lsm_se;
    }
    for (int i = 0; i < d; ++i) {
      for (int64_t p = 0; p < P; ++p) tmp[p] = vv[(size_t)p * d + i];
      mean_se(tmp, P, &vega_v0[i], &vega_v0_se[i], NULL);
      for (int64_t p = 0; p < P; ++p) tmp[p] = vt[(size_t)p * d + i];
      mean_se(tmp, P, &vega_theta[i], &vega_theta_se[i], NULL);
    }
    for (int i = 0; i < d; ++i) {
      dcorr[i * d + i] = 0.0;
      dcorr_se[i * d + i] = 0.0;
      for (int j = 0; j < i; ++j) {
        const int q = i * (i - 1) / 2 + j;
        for (int64_t p = 0; p < P; ++p) tmp[p] = dc[(size_t)p * npair + q];
        mean_se(tmp, P, &dcorr[i * d + j], &dcorr_se[i * d + j], NULL);
        dcorr[j * d + i] = dcorr[i * d + j];
        dcorr_se[j * d + i] = dcorr_se[i * d + j];
      }
    }
  }
  free(tau); free(dL); free(val); free(vv); free(vt); free(dc); free(tmp);
  return rc;
}

typedef struct {
  const basket_setup* S;
  const int32_t* tau;
  double* out;
} bstop_ctx;

static void bstop_range(void* vctx, int64_t bgn, int64_t end) {
  bstop_ctx* c = (bstop_ctx*)vctx;
  const ref_basket* b = c->S->b;
  for (int64_t p = bgn; p < end; ++p) {
    double x[REF_MAX_ASSETS], v[REF_MAX_ASSETS];
    basket_init_state(b, x, v);
    for (int32_t n = 0; n < c->tau[p]; ++n) basket_transition(c->S, p, n, x, v, NULL, NULL);
    c->out[p] = exp(-b->r * (c->S->dt * c->tau[p])) * basket_intrinsic(b, basket_value(b, x));
  }
}

int ref_basket_stopped_values(const ref_basket* b, const int32_t* tau, int nthreads, double* out) {
  basket_setup S;
  if (!tau || !out || basket_setup_init(b, &S)) return -1;
  for (int64_t p = 0; p < b->paths; ++p)
    if (tau[p] < 0 || tau[p] > b->steps) return -1;
  bstop_ctx c = {&S, tau, out};
  parallel_range(b->paths, nthreads, bstop_range, &c);
  return 0;
}

/* ------------------------------------------------------------------------- */
/* Broadie-Kaya exact simulation (Broadie and Kaya 2006).                     */
/* ------------------------------------------------------------------------- */

/* Legendre's continued fraction for the upper incomplete gamma function,
 *   Gamma(a, x) = x^a e^{-x} / (b_0 + a_1/(b_1 + a_2/(b_2 + ...))),  b_j = x + 2j + 1 - a,
 *   a_j = -j (j - a)  (DLMF 8.9.2 in its even contraction),
 * evaluated plainly: the fraction cut at depth M is summed from the bottom up, and M doubles
 * until two depths agree to 1e-15.  Used where it converges quickly, x >= a + 1. */
static double upper_gamma_fraction(double a, double x) {
  double prev = 0.0;
  for (int M = 16; M <= (1 << 20); M *= 2) {
    double g = x + 2.0 * M + 1.0 - a;
    for (int j = M; j >= 1; --j) g = (x + 2.0 * (j - 1) + 1.0 - a) + (-(double)j * (j - a)) / g;
    if (M > 16 && fabs(g - prev) <= 1e-15 * fabs(g)) return g;
    prev = g;
  }
  return prev;
}

/* Regularised lower incomplete gamma P(a, x) = gamma(a, x) / Gamma(a).  For x < a + 1 its power
 * series P(a, x) = sum_k x^(a+k) e^{-x} / Gamma(a + k + 1) (DLMF 8.7.1): the k = 0 term from
 * lgamma, each next one x / (a + k) times the last; the terms decrease, so the sum stops once a
 * term no longer changes it.  Otherwise 1 - Gamma(a, x) / Gamma(a) with the continued fraction
 * above. */
static double inc_gamma_p(double a, double x) {
  if (x <= 0.0) return 0.0;
  if (x < a + 1.0) {
    double term = exp(a * log(x) - x - lgamma(a + 1.0)), sum = term;
    for (int k = 1; k < 100000 && term > 1e-17 * sum; ++k) {
      term *= x / (a + k);
      sum += term;
    }
    return sum;
  }
  return 1.0 - exp(a * log(x) - x - lgamma(a)) / upper_gamma_fraction(a, x);
}

/* CDF and density of V = c X, X noncentral chi-square with df degrees of freedom and
 * noncentrality lam, as the Poisson(lam / 2) mixture of central chi-squares. */
static void ncx2_cdf_pdf(double v, double c, double df, double lam, double* F, double* f) {
  const double y = v / (2.0 * c);
  const double m = 0.5 * lam;
  int jlo = 0, jhi = 0;
  if (m > 0.0) {
    const double sd = sqrt(m);
    jlo = (int)fmax(0.0, floor(m - 12.0 * sd - 10.0));
    jhi = (int)ceil(m + 12.0 * sd + 10.0);
  }
  double s = 0.0, sp = 0.0;
  for (int j = jlo; j <= jhi; ++j) {
    const double lw = (m > 0.0) ? (-m + j * log(m) - lgamma(j + 1.0)) : (j == 0 ? 0.0 : -INFINITY);
    const double w = exp(lw);
    if (w == 0.0) continue;
    const double a = 0.5 * df + j;
    s += w * inc_gamma_p(a, y);
    if (y > 0.0) sp += w * exp((a - 1.0) * log(y) - y - lgamma(a));
  }
  *F = s;
  *f = sp / (2.0 * c);
}

double ref_bk_variance(double v, double kappa, double theta, double xi, double dt, double u) {
  const double E = exp(-kappa * dt);
  if (!(xi > 0.0)) return theta + (v - theta) * E;
  const double c = xi * xi * (1.0 - E) / (4.0 * kappa);
  const double df = 4.0 * kappa * theta / (xi * xi);
  const double lam = v * E / c;
  /* safeguarded Newton on F(e^y) = u in y = ln V (relative precision at any scale), bracketed
   * by [ln 1e-300, ln(mean + 40 sd)] */
  const double mean = c * (df + lam), sd = c * sqrt(2.0 * (df + 2.0 * lam));
  double lo = log(1e-300), hi = log(mean + 40.0 * sd);
  double y = log(mean);
  for (int it = 0; it < 400; ++it) {
    const double x = exp(y);
    double F, f;
    ncx2_cdf_pdf(x, c, df, lam, &F, &f);
    if (F < u) lo = y; else hi = y;
    double yn = (f * x > 0.0) ? y - (F - u) / (f * x) : 0.5 * (lo + hi);
    if (!(yn > lo && yn < hi)) yn = 0.5 * (lo + hi);
    if (fabs(yn - y) <= 1e-14 || hi - lo <= 1e-14) return exp(yn);
    y = yn;
  }
  return exp(y);
}

/* ln of the modified Bessel series S(z) = sum_k (z^2 / 4)^k / (k! Gamma(k + nu + 1)), so that
 * I_nu(z) = (z / 2)^nu S(z); summed with the terms scaled by e^{-|z|} against overflow. */
static double complex log_bessel_series(double complex z, double nu) {
  const double az = cabs(z);
  const double complex q = 0.25 * z * z;
  double complex t = cexp(-az - lgamma(nu + 1.0) + 0.0 * I), s = t;
  for (int k = 1; k < 100000; ++k) {
    t *= q / ((double)k * (k + nu));
    s += t;
    if (k > az && cabs(t) < 1e-18 * cabs(s)) break;
  }
  return az + clog(s);
}

/* ln of the characteristic function E[exp(i a I) | v_u, v_t] of I = integral of V over one
 * step (Broadie and Kaya, from the Bessel-bridge law of the CIR process).  With
 * g = sqrt(kappa^2 - 2 xi^2 i a):
 *   g e^{-(g - kappa) dt/2} (1 - e^{-kappa dt}) / (kappa (1 - e^{-g dt}))
 *   * exp{(v_u + v_t)/xi^2 [kappa (1 + e^{-kappa dt})/(1 - e^{-kappa dt}) - g (1 + e^{-g dt})/(1 - e^{-g dt})]}
 *   * I_nu(z(g)) / I_nu(z(kappa)),  z(g) = sqrt(v_u v_t) 4 g e^{-g dt/2} / (xi^2 (1 - e^{-g dt})),
 * nu = 2 kappa theta / xi^2 - 1.  ln(z(g) / z(kappa)) is summed from principal logarithms of
 * g / kappa and of 1 - e^{-g dt} (both of positive real part), so it is continuous in a. */
static double complex bk_log_cf(double a, double vu, double vt, double kappa, double theta, double xi, double dt) {
  const double complex g = csqrt(kappa * kappa - 2.0 * xi * xi * a * I);
  const double ek = exp(-kappa * dt);
  const double complex eg = cexp(-g * dt);
  const double nu = 2.0 * kappa * theta / (xi * xi) - 1.0;
  const double complex lratio = clog(g / kappa) - 0.5 * (g - kappa) * dt + log(1.0 - ek) - clog(1.0 - eg);
  double complex l = lratio;  /* the first factor equals z(g) / z(kappa) */
  l += (vu + vt) / (xi * xi) * (kappa * (1.0 + ek) / (1.0 - ek) - g * (1.0 + eg) / (1.0 - eg));
  l += nu * lratio;  /* I_nu(z) / I_nu(z0) = (z / z0)^nu S(z) / S(z0); S -> 1 / Gamma(nu + 1) at 0 */
  if (vu > 0.0 && vt > 0.0) {
    const double z0 = sqrt(vu * vt) * 4.0 * kappa * exp(-0.5 * kappa * dt) / (xi * xi * (1.0 - ek));
    const double complex z = z0 * cexp(lratio);
    l += log_bessel_series(z, nu) - creal(log_bessel_series(z0 + 0.0 * I, nu));
  }
  return l;
}

double ref_bk_log_cf_re(double a, double vu, double vt, double kappa, double theta, double xi, double dt) {
  return creal(bk_log_cf(a, vu, vt, kappa, theta, xi, dt));
}
double ref_bk_log_cf_im(double a, double vu, double vt, double kappa, double theta, double xi, double dt) {
  return cimag(bk_log_cf(a, vu, vt, kappa, theta, xi, dt));
}

double ref_bk_integrated_variance(double vu, double vt, double kappa, double theta, double xi, double dt,
                                  double u) {
  if (!(xi > 0.0)) return theta * dt + (vu - theta) * (1.0 - exp(-kappa * dt)) / kappa;
  /* mean and variance from the characteristic function near 0, for the Fourier grid */
  const double guess = 0.5 * (vu + vt) * dt + 1e-12;
  const double ea = 1e-4 / guess;
  const double complex p = cexp(bk_log_cf(ea, vu, vt, kappa, theta, xi, dt));
  const double mu = cimag(p) / ea;
  const double m2 = 2.0 * (1.0 - creal(p)) / (ea * ea);
  const double sd = sqrt(fmax(m2 - mu * mu, 1e-6 * mu * mu));
  /* F(x) = h x / pi + (2 / pi) sum_j sin(h j x) / j Re phi(h j): the trapezoid rule for the
   * Fourier inversion of the CDF.  Its error at x is about the mass beyond 2 pi / h - x, so the
   * period is twice u_e = mu + 20 sd and the draws stay in [0, u_e]. */
  const double ue = mu + 20.0 * sd;
  const double h = M_PI / ue;
  enum { JMAX = 20000 };
  static __thread double rephi[JMAX + 1];
  int M = 0;
  for (int j = 1; j <= JMAX; ++j) {
    const double complex ph = cexp(bk_log_cf(h * j, vu, vt, kappa, theta, xi, dt));
    rephi[j] = creal(ph);
    M = j;
    if (cabs(ph) / j < M_PI * 1e-13 / 2.0) break;
  }
  double lo = 0.0, hi = ue, x = mu;
  for (int it = 0; it < 200; ++it) {
    double F = h * x / M_PI, f = h / M_PI;
    for (int j = 1; j <= M; ++j) {
      F += 2.0 / M_PI * sin(h * j * x) / j * rephi[j];
      f += 2.0 * h / M_PI * cos(h * j * x) * rephi[j];
    }
    if (F < u) lo = x; else hi = x;
    double xn = (f > 0.0) ? x - (F - u) / f : 0.5 * (lo + hi);
    if (!(xn > lo && xn < hi)) xn = 0.5 * (lo + hi);
    if (fabs(xn - x) <= 1e-13 * mu || hi - lo <= 1e-14 * mu) return xn;
    x = xn;
  }
  return x;
}

void ref_bk_step(double* x, double* v, double r, double kappa, double theta, double xi, double rho, double dt,
                 double z2, double u_v, double u_i) {
  const double vu = *v;
  const double vt = ref_bk_variance(vu, kappa, theta, xi, dt, u_v);
  const double iv = ref_bk_integrated_variance(vu, vt, kappa, theta, xi, dt, u_i);
  /* the variance noise integral from the CIR equation; absent when xi = 0 (rho taken as 0) */
  const double wv = (xi > 0.0) ? (vt - vu - kappa * theta * dt + kappa * iv) / xi : 0.0;
  const double rh = (xi > 0.0) ? rho : 0.0;
  *x = *x + r * dt - 0.5 * iv + rh * wv + sqrt((1.0 - rh * rh) * iv) * z2;
  *v = vt;
}
