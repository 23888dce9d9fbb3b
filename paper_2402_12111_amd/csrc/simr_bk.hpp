// simr_bk.hpp -- Broadie and Kaya's exact simulation of one Heston step, in FP64 device code.
//
//   V_t | v_u   = c X, X noncentral chi-square (4 kappa theta / xi^2 degrees of freedom,
//                 noncentrality v_u e^{-kappa dt} / c, c = xi^2 (1 - e^{-kappa dt}) / (4 kappa)),
//                 drawn by inverting its Poisson-mixture CDF at the uniform of word 2;
//   I | v_u, V_t  the integrated variance, drawn by inverting at the uniform of word 3 the CDF
//                 that the trapezoid rule gives from the conditional characteristic function
//                 (the Bessel-bridge law of the CIR process);
//   x_t = x_u + r dt - I / 2 + rho (V_t - v_u - kappa theta dt + kappa I) / xi
//         + sqrt((1 - rho^2) I) Z2.
// xi = 0: the deterministic CIR mean and its exact integral (rho taken as 0).  The FP32 path
// state is widened to FP64 for the step and rounded back.  The series for the Bessel function
// keeps full accuracy while its argument stays moderate (few large steps: the scheme's use as
// an accuracy reference); roots are found to ~1e-13 relative.
#pragma once

#include <hip/hip_runtime.h>

namespace simr {
namespace bk {

struct cplx {
  double re, im;
};
__device__ __forceinline__ cplx cx(double re, double im = 0.0) { return cplx{re, im}; }
__device__ __forceinline__ cplx operator+(cplx a, cplx b) { return cx(a.re + b.re, a.im + b.im); }
__device__ __forceinline__ cplx operator-(cplx a, cplx b) { return cx(a.re - b.re, a.im - b.im); }
__device__ __forceinline__ cplx operator*(cplx a, cplx b) {
  return cx(a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re);
}
__device__ __forceinline__ cplx operator*(double s, cplx a) { return cx(s * a.re, s * a.im); }
__device__ __forceinline__ cplx cdiv(cplx a, cplx b) {  // scaled to avoid overflow
  const double s = fmax(fabs(b.re), fabs(b.im));
  const double br = b.re / s, bi = b.im / s;
  const double d = br * br + bi * bi;
  return cx((a.re * br + a.im * bi) / (s * d), (a.im * br - a.re * bi) / (s * d));
}
__device__ __forceinline__ double cabs_(cplx a) { return hypot(a.re, a.im); }
__device__ __forceinline__ cplx cexp_(cplx a) {
  const double m = exp(a.re);
  double s, c;
  sincos(a.im, &s, &c);
  return cx(m * c, m * s);
}
__device__ __forceinline__ cplx clog_(cplx a) { return cx(log(cabs_(a)), atan2(a.im, a.re)); }
__device__ __forceinline__ cplx csqrt_(cplx a) {  // principal branch (non-negative real part)
  const double m = cabs_(a);
  const double re = sqrt(0.5 * (m + a.re));
  const double im = sqrt(fmax(0.5 * (m - a.re), 0.0));
  return cx(re, a.im < 0.0 ? -im : im);
}

// Regularised lower incomplete gamma P(a, x).  Below x = a + 1 the power series
//   P = x^a e^{-x} / Gamma(a + 1) * sum_k x^k / ((a + 1)(a + 2)...(a + k)).
// Above it P = 1 - Q, with the upper function Q = x^a e^{-x} / (Gamma(a) g) and g the continued
// fraction g = b_0 + a_1/(b_1 + a_2/(b_2 + ...)), b_j = x + 2j + 1 - a, a_j = -j (j - a)
// (Legendre's fraction for the upper incomplete gamma function, in its even contraction).  g is
// evaluated front to back by the modified Lentz algorithm (W. J. Lentz, Applied Optics 15, 1976;
// I. J. Thompson and A. R. Barnett, J. Comput. Phys. 64, 1986): f_j = f_{j-1} C_j D_j with
// C_j = b_j + a_j / C_{j-1} and D_j = 1 / (b_j + a_j D_{j-1}), starting from f_0 = C_0 = b_0,
// D_0 = 0, any zero denominator replaced by a tiny number, until C_j D_j is 1 to rounding.
__device__ inline double inc_gamma_p(double a, double x) {
  if (!(x > 0.0)) return 0.0;
  const double log_pref = a * log(x) - x - lgamma(a);  // ln(x^a e^{-x} / Gamma(a))
  if (x < a + 1.0) {
    double ratio = 1.0, total = 1.0;  // k = 0 term of the sum; the 1/a goes into the prefactor
    for (int k = 1; k < 20000; ++k) {  // a + k > x after at most ~x terms; bounded regardless
      ratio *= x / (a + (double)k);
      total += ratio;
      if (ratio < total * 1e-17) break;
    }
    return total * exp(log_pref) / a;
  }
  constexpr double kTiny = 1e-300;
  const double b0 = x + 1.0 - a;
  double f = fabs(b0) < kTiny ? kTiny : b0;
  double C = f, D = 0.0;
  for (int j = 1; j < 20000; ++j) {
    const double aj = -(double)j * ((double)j - a);
    const double bj = b0 + 2.0 * (double)j;
    D = bj + aj * D;
    D = 1.0 / (fabs(D) < kTiny ? kTiny : D);
    C = bj + aj / C;
    if (fabs(C) < kTiny) C = kTiny;
    const double step = C * D;
    f *= step;
    if (fabs(step - 1.0) < 1e-16) break;
  }
  return 1.0 - exp(log_pref) / f;
}

// CDF F and density f at v of c X, X noncentral chi-square(df, lam): Poisson(lam / 2) weights
// over central chi-squares, the mixture truncated 12 standard deviations either side.
__device__ inline void ncx2_cdf_pdf(double v, double c, double df, double lam, double& F, double& f) {
  const double y = v / (2.0 * c);
  const double m = 0.5 * lam;
  int jlo = 0, jhi = 0;
  if (m > 0.0) {
    const double sd = sqrt(m);
    jlo = (int)fmax(0.0, floor(m - 12.0 * sd - 10.0));
    jhi = (int)ceil(m + 12.0 * sd + 10.0);
  }
  const double lm = m > 0.0 ? log(m) : 0.0;
  double s = 0.0, sp = 0.0;
  for (int j = jlo; j <= jhi; ++j) {
    const double w = m > 0.0 ? exp(-m + (double)j * lm - lgamma((double)j + 1.0)) : 1.0;
    const double a = 0.5 * df + (double)j;
    s += w * inc_gamma_p(a, y);
    if (y > 0.0) sp += w * exp((a - 1.0) * log(y) - y - lgamma(a));
  }
  F = s;
  f = sp / (2.0 * c);
}

// The exact variance draw: safeguarded Newton on F(e^y) = u in y = ln V.
__device__ inline double variance(double v, double kappa, double theta, double xi, double dt, double u) {
  const double E = exp(-kappa * dt);
  if (!(xi > 0.0)) return theta + (v - theta) * E;
  const double c = xi * xi * (1.0 - E) / (4.0 * kappa);
  const double df = 4.0 * kappa * theta / (xi * xi);
  const double lam = v * E / c;
  const double mean = c * (df + lam), sd = c * sqrt(2.0 * (df + 2.0 * lam));
  double lo = log(1e-300), hi = log(mean + 40.0 * sd), y = log(mean);
  for (int it = 0; it < 200; ++it) {
    const double x = exp(y);
    double F, f;
    ncx2_cdf_pdf(x, c, df, lam, F, f);
    if (F < u) lo = y; else hi = y;
    double yn = (f * x > 0.0) ? y - (F - u) / (f * x) : 0.5 * (lo + hi);
    if (!(yn > lo && yn < hi)) yn = 0.5 * (lo + hi);
    if (fabs(yn - y) <= 1e-14 || hi - lo <= 1e-14) return exp(yn);
    y = yn;
  }
  return exp(y);
}

// ln S(z), S(z) = sum_k (z^2/4)^k / (k! Gamma(k + nu + 1)) (I_nu(z) = (z/2)^nu S(z)), the terms
// scaled by e^{-|z|}.
__device__ inline cplx log_bessel_series(cplx z, double nu) {
  const double az = cabs_(z);
  const cplx q = 0.25 * (z * z);
  cplx t = cx(exp(-az - lgamma(nu + 1.0))), s = t;
  const int kmax = (int)fmin(4.0 * az, 1e6) + 2000;  // bounded also for non-finite input
  for (int k = 1; k < kmax; ++k) {
    const double den = (double)k * ((double)k + nu);
    t = cx((t.re * q.re - t.im * q.im) / den, (t.re * q.im + t.im * q.re) / den);
    s = s + t;
    const double at = cabs_(t);
    if (((double)k > az && at < 1e-18 * cabs_(s)) || !(at == at)) break;
  }
  return cx(az) + clog_(s);
}

// ln E[exp(i a I) | v_u, v_t]: with g = sqrt(kappa^2 - 2 xi^2 i a) and the ratio
// r = z(g) / z(kappa) = (g / kappa) e^{-(g - kappa) dt / 2} (1 - e^{-kappa dt}) / (1 - e^{-g dt})
// (its logarithm summed from principal logarithms of factors with positive real part, so the
// phase is continuous in a):  ln r + (v_u + v_t) / xi^2 [kappa coth-term - g coth-term]
// + nu ln r + ln S(z0 r) - ln S(z0).
struct CfConst {
  double kappa, xi, dt, nu, ek, ckap, z0, ls0, vs;
};

__device__ inline cplx log_cf(const CfConst& k, double a) {
  const cplx g = csqrt_(cx(k.kappa * k.kappa, -2.0 * k.xi * k.xi * a));
  const cplx eg = cexp_(cx(-g.re * k.dt, -g.im * k.dt));
  const cplx one_m_eg = cx(1.0 - eg.re, -eg.im);
  const cplx lr = clog_(cx(g.re / k.kappa, g.im / k.kappa)) - cx(0.5 * (g.re - k.kappa) * k.dt, 0.5 * g.im * k.dt) +
                  cx(log(1.0 - k.ek)) - clog_(one_m_eg);
  const cplx coth_g = cdiv(g * cx(1.0 + eg.re, eg.im), one_m_eg);
  cplx l = (1.0 + k.nu) * lr + (k.vs / (k.xi * k.xi)) * (cx(k.ckap) - coth_g);
  if (k.z0 > 0.0) l = l + log_bessel_series(k.z0 * cexp_(lr), k.nu) - cx(k.ls0);
  return l;
}

// The integrated-variance draw: Newton (safeguarded by bisection on [0, u_e]) on the trapezoid
// CDF F(x) = h x / pi + (2 / pi) sum_{j=1..M} sin(h j x) / j Re phi(h j), period 2 pi / h = 2 u_e,
// u_e = mu + 20 sd from the characteristic function near 0, M where |phi(h j)| / j < pi 1e-13 / 2.
__device__ inline double integrated_variance(double vu, double vt, double kappa, double theta, double xi,
                                             double dt, double u) {
  if (!(xi > 0.0)) return theta * dt + (vu - theta) * (1.0 - exp(-kappa * dt)) / kappa;
  CfConst k;
  k.kappa = kappa;
  k.xi = xi;
  k.dt = dt;
  k.nu = 2.0 * kappa * theta / (xi * xi) - 1.0;
  k.ek = exp(-kappa * dt);
  k.ckap = kappa * (1.0 + k.ek) / (1.0 - k.ek);
  k.vs = vu + vt;
  k.z0 = (vu > 0.0 && vt > 0.0) ? sqrt(vu * vt) * 4.0 * kappa * exp(-0.5 * kappa * dt) / (xi * xi * (1.0 - k.ek))
                                : 0.0;
  k.ls0 = k.z0 > 0.0 ? log_bessel_series(cx(k.z0), k.nu).re : 0.0;
  const double guess = 0.5 * (vu + vt) * dt + 1e-12;
  const double ea = 1e-4 / guess;
  const cplx p = cexp_(log_cf(k, ea));
  const double mu = p.im / ea;
  const double m2 = 2.0 * (1.0 - p.re) / (ea * ea);
  const double sd = sqrt(fmax(m2 - mu * mu, 1e-6 * mu * mu));
  if (!(mu > 0.0) || !(sd < 1e300)) return guess;  // no usable moments: the trapezoid value
  const double ue = mu + 20.0 * sd;
  const double h = M_PI / ue;
  int M = 1;
  for (; M < 4096; ++M) {
    const cplx l = log_cf(k, h * M);
    if (exp(l.re) / (double)M < M_PI * 1e-13 / 2.0) break;
  }
  double lo = 0.0, hi = ue, x = mu;
  for (int it = 0; it < 100; ++it) {  // bisection alone reaches 1e-14 mu in about 50 steps
    double F = h * x / M_PI, f = h / M_PI;
    for (int j = 1; j <= M; ++j) {
      const double re = cexp_(log_cf(k, h * j)).re;
      double s, c;
      sincos(h * j * x, &s, &c);
      F += 2.0 / M_PI * s / (double)j * re;
      f += 2.0 * h / M_PI * c * re;
    }
    if (F < u) lo = x; else hi = x;
    double xn = (f > 0.0) ? x - (F - u) / f : 0.5 * (lo + hi);
    if (!(xn > lo && xn < hi)) xn = 0.5 * (lo + hi);
    if (fabs(xn - x) <= 1e-13 * mu || hi - lo <= 1e-14 * mu) return xn;
    x = xn;
  }
  return x;
}

}  // namespace bk
}  // namespace simr
