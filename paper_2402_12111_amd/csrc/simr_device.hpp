// simr_device.hpp -- device building blocks of the Heston Monte Carlo hot path on
// gfx950: counter-based random words, the Gaussian transform, the QE and
// full-truncation Euler transitions, compensated sums and wave64 / block
// reductions.  One path per lane, all path state in registers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "simr_bk.hpp"

namespace simr {

constexpr int kWave = 64;

// Global-memory (address space 1) view of a pointer that reaches a kernel inside a struct.  A
// generic pointer compiles to FLAT memory instructions, which count on the LDS counter as well
// as the vector-memory one, so every LDS wait (each block barrier) also waits for the FLAT
// loads still in flight.  Through this view the accesses are global loads and stores with a
// scalar base and a 32-bit vector offset where the index allows it.
#define SIMR_GLOBAL __attribute__((address_space(1)))
template <class T>
__device__ __forceinline__ const SIMR_GLOBAL T* as_global(const T* p) {
  return (const SIMR_GLOBAL T*)p;
}
template <class T>
__device__ __forceinline__ SIMR_GLOBAL T* as_global(T* p) {
  return (SIMR_GLOBAL T*)p;
}

// ---------------------------------------------------------------------------------------------
// Per-option constants, computed in FP64 on the host and rounded once to FP32.
// ---------------------------------------------------------------------------------------------
struct DevOpt {
  // QE variance step (Andersen 2008): m = theta + (v - theta) E, s^2 = v A1 + A2
  float E, A1, A2, theta;
  // QE log-price step: x += C0 + K1 v + K2 V + sqrt(K3 v + K4 V) Z2, C0 = r dt + K0;
  // martingale correction: A = K2 + K4 / 2 and K13 = K1 + K3 / 2 (K0* = -ln E[e^{A V}] - K13 v)
  float C0, K1, K2, K3, K4, Amg, K13;
  // full-truncation Euler: v += kthdt - kdt v+ + xisdt sqrt(v+) Z1,
  //                        x += rdt - hdt v+ + sdt sqrt(v+) (rho Z1 + srho Z2)
  float kdt, kthdt, xisdt, sdt, hdt, rdt, rho, srho;
  // contract
  float S0, K, disc, v0, invK, invTheta;
  // adjoint chain rule: derivatives of the step constants w.r.t. the model parameters
  float dE_dk, dA1_dk, dA1_dxi, dA2_dth, dA2_dk, dA2_dxi;
  float dC0_dth, dC0_dr, dC0_dk, dC0_dxi, dC0_drho;
  float dK1_dk, dK1_dxi, dK1_drho, dK2_dk, dK2_dxi, dK2_drho, dK3_drho, dK4_drho;
  // derivatives in the maturity T with the step count fixed (dt = T / N); rN = r / N
  float dE_dT, dA1_dT, dA2_dT, dC0_dT, dK1_dT, dK2_dT, dK3_dT, rN;
  // the same for the full-truncation Euler constants rdt, hdt, sdt, kdt, kthdt, xisdt
  float fdT_rdt, fdT_hdt, fdT_sdt, fdT_kdt, fdT_kthdt, fdT_xisdt;
  float dt;
  // truncated Gaussian scheme: (mu / m, log2(sigma / m)) at log2(psi) = kTgLo + i h, i < kTgN,
  // then their derivatives in log2(psi) at the same nodes (device table of 2 kTgN entries)
  const float2* tg;
  int32_t payoff;     // simr_payoff
  int32_t steps;
  int32_t paths;
  uint32_t stream;
  uint32_t seed_lo, seed_hi;
  int32_t slot0;      // first partial-sum slot of this option (batch)
  int32_t ntiles;     // path tiles of this option (batch)
  // Broadie-Kaya exact scheme: the model in FP64
  double bk_kappa, bk_theta, bk_xi, bk_rho, bk_r, bk_dt;
};

// ---------------------------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11).  Counter (c0, c1, c2, c3) = (step, path,
// stream, 0), key = seed.  Only c1 differs between lanes, so the first rounds work mostly on
// wave-uniform words and the compiler keeps them on the scalar unit.
// ---------------------------------------------------------------------------------------------
struct Words { uint32_t w0, w1, w2, w3; };

// a ^ b ^ c in one gfx950 VALU instruction (v_bitop3_b32 with truth table 0x96).
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c) {
  return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}

__device__ __forceinline__ Words philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                               uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int round = 0; round < 10; ++round) {
    const uint64_t pa = (uint64_t)0xD2511F53u * c0;   // one v_mad_u64_u32 gives hi and lo
    const uint64_t pb = (uint64_t)0xCD9E8D57u * c2;
    // the first two rounds still mix wave-uniform words (kept on the scalar unit by plain XORs);
    // from the third on every word differs between lanes: one 3-input VALU op per word
    const uint32_t n0 = round < 2 ? (uint32_t)(pb >> 32) ^ c1 ^ k0 : xor3((uint32_t)(pb >> 32), c1, k0);
    const uint32_t n2 = round < 2 ? (uint32_t)(pa >> 32) ^ c3 ^ k1 : xor3((uint32_t)(pa >> 32), c3, k1);
    c1 = (uint32_t)pb;
    c3 = (uint32_t)pa;
    c0 = n0;
    c2 = n2;
    k0 += 0x9E3779B9u;  // Weyl key schedule; the bump after the last round is unused
    k1 += 0xBB67AE85u;
  }
  return Words{c0, c1, c2, c3};
}

// ((w >> 9) + 1/2) * 2^-23: the odd multiples of 2^-24 in (0,1), exact in FP32 (and 1 - u too).
__device__ __forceinline__ float u01(uint32_t w) {
  return __builtin_fmaf((float)(w >> 9), 0x1p-23f, 0x1p-24f);
}

// Box-Muller with the hardware transcendentals: v_log_f32 is log2, and v_sin_f32 / v_cos_f32
// take their argument in revolutions, so sin(2 pi u) needs no multiply and no range reduction.
__device__ __forceinline__ void box_muller(float u0, float u1, float& z1, float& z2) {
  const float r = __builtin_amdgcn_sqrtf(__builtin_amdgcn_logf(u0) * -1.38629436111989061883f);  // -2 ln 2
  z1 = r * __builtin_amdgcn_cosf(u1);
  z2 = r * __builtin_amdgcn_sinf(u1);
}

__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ float fsqrt(float x) { return __builtin_amdgcn_sqrtf(x); }

// The variates of transition n of path p (u2, from word 3, is drawn by the Broadie-Kaya scheme
// only).
struct Draw { float z1, z2, u, u2; };
__device__ __forceinline__ Draw draw(const DevOpt& o, uint32_t n, uint32_t path) {
  const Words w = philox4x32_10(n, path, o.stream, 0u, o.seed_lo, o.seed_hi);
  Draw d;
  box_muller(u01(w.w0), u01(w.w1), d.z1, d.z2);
  d.u = u01(w.w2);
  d.u2 = u01(w.w3);
  return d;
}

// ---------------------------------------------------------------------------------------------
// VariancePathQE: Andersen's QE step, psi_c = 1.5.
// ---------------------------------------------------------------------------------------------
constexpr float kPsiC = 1.5f;

__device__ __forceinline__ float qe_variance(const DevOpt& o, float v, float z1, float u) {
  const float m = __builtin_fmaf(v - o.theta, o.E, o.theta);
  const float s2 = __builtin_fmaf(v, o.A1, o.A2);
  if (!(s2 > 0.0f)) return m;  // xi = 0: deterministic variance
  const float m2 = m * m;
  const float psi = s2 * rcp(m2);
  float V;
  if (psi <= kPsiC) {
    const float t = 2.0f * m2 * rcp(s2);                   // 2 / psi
    const float b2 = (t - 1.0f) + fsqrt(t * (t - 1.0f));
    const float b = fsqrt(b2);
    const float a = m * rcp(1.0f + b2);
    const float bz = b + z1;
    V = a * (bz * bz);
  } else {
    const float p = (psi - 1.0f) * rcp(psi + 1.0f);
    const float omp = 1.0f - p;
    // ln((1-p)/(1-u)) * m / (1-p); zero mass for u <= p
    const float L = __builtin_amdgcn_logf(omp * rcp(1.0f - u)) * 0.69314718055994530942f;
    V = (u <= p) ? 0.0f : L * m * rcp(omp);
  }
  return V;
}

// LogPricePathQE: x_{n+1} = x_n + C0 + K1 v + K2 V + sqrt(K3 v + K4 V) Z2.
__device__ __forceinline__ float qe_logprice_inc(const DevOpt& o, float v, float V, float z2) {
  const float w = __builtin_fmaf(o.K3, v, o.K4 * V);
  float inc = __builtin_fmaf(o.K2, V, __builtin_fmaf(o.K1, v, o.C0));
  return __builtin_fmaf(fsqrt(w), z2, inc);
}

// The variance part of the full-truncation Euler transition (the same expression as fte_step).
__device__ __forceinline__ float fte_variance(const DevOpt& o, float v, float z1) {
  const float vp = fmaxf(v, 0.0f);
  const float sv = fsqrt(vp);
  return v + __builtin_fmaf(-o.kdt, vp, o.kthdt) + o.xisdt * sv * z1;
}

// Full-truncation Euler transition of (x, v).
__device__ __forceinline__ void fte_step(const DevOpt& o, float& x, float& v, float z1, float z2) {
  const float vp = fmaxf(v, 0.0f);
  const float sv = fsqrt(vp);
  const float vn = v + __builtin_fmaf(-o.kdt, vp, o.kthdt) + o.xisdt * sv * z1;
  const float zs = __builtin_fmaf(o.rho, z1, o.srho * z2);
  x += __builtin_fmaf(-o.hdt, vp, o.rdt) + o.sdt * sv * zs;
  v = vn;
}

// The QE variance step together with g = ln E[exp(A V) | v] of the branch it takes (Andersen's
// martingale correction): quadratic branch A b^2 a / (1 - 2 A a) - ln(1 - 2 A a) / 2, exponential
// branch ln(p + beta (1 - p) / (beta - A)), deterministic variance A m.  ok = false where the
// moment does not exist (2 A a >= 1, or A >= beta).
__device__ __forceinline__ float qe_variance_mgf(const DevOpt& o, float v, float z1, float u, float& g, bool& ok) {
  const float A = o.Amg;
  const float m = __builtin_fmaf(v - o.theta, o.E, o.theta);
  const float s2 = __builtin_fmaf(v, o.A1, o.A2);
  ok = true;
  if (!(s2 > 0.0f)) {
    g = A * m;
    return m;
  }
  const float m2 = m * m;
  const float psi = s2 * rcp(m2);
  constexpr float kLn2 = 0.69314718055994530942f;
  float V;
  if (psi <= kPsiC) {
    const float t = 2.0f * m2 * rcp(s2);
    const float b2 = (t - 1.0f) + fsqrt(t * (t - 1.0f));
    const float b = fsqrt(b2);
    const float a = m * rcp(1.0f + b2);
    const float bz = b + z1;
    V = a * (bz * bz);
    const float dd = __builtin_fmaf(-2.0f * A, a, 1.0f);
    ok = dd > 0.0f;
    g = A * b2 * a * rcp(dd) - 0.5f * kLn2 * __builtin_amdgcn_logf(dd);
  } else {
    const float p = (psi - 1.0f) * rcp(psi + 1.0f);
    const float omp = 1.0f - p;
    const float L = __builtin_amdgcn_logf(omp * rcp(1.0f - u)) * kLn2;
    V = (u <= p) ? 0.0f : L * m * rcp(omp);
    const float beta = omp * rcp(m);
    ok = A < beta;
    g = kLn2 * __builtin_amdgcn_logf(__builtin_fmaf(beta * omp, rcp(beta - A), p));
  }
  return V;
}

// ---------------------------------------------------------------------------------------------
// Andersen's truncated Gaussian variance step: V = max(mu + sigma Z1, 0) with mu / m and sigma / m
// functions of psi alone (moment matching of the CIR transition), read from a table uniform in
// log2(psi) and interpolated linearly (sigma / m in the log domain).  Below the table r = mu /
// sigma exceeds 8, the truncation terms Phi(-r) and phi(r) are below 1e-14 and the step is the
// untruncated m (1 + sqrt(psi) Z1); above it (psi > 2^14: Feller ratio 2 kappa theta / xi^2
// below about 1e-4) the last entry holds.
// ---------------------------------------------------------------------------------------------
constexpr int kTgN = 8192;
constexpr float kTgLo = -6.0f, kTgHi = 14.0f;
constexpr float kTgInvH = (float)(kTgN - 1) / (kTgHi - kTgLo);

__device__ __forceinline__ float tg_variance(const DevOpt& o, float v, float z1) {
  const float m = __builtin_fmaf(v - o.theta, o.E, o.theta);
  const float s2 = __builtin_fmaf(v, o.A1, o.A2);
  if (!(s2 > 0.0f)) return m;  // xi = 0: deterministic variance
  const float psi = s2 * rcp(m * m);
  const float lp = __builtin_amdgcn_logf(psi);  // log2
  float fm, fs;
  if (lp < kTgLo) {
    fm = 1.0f;
    fs = fsqrt(psi);
  } else {
    const float t = fminf((lp - kTgLo) * kTgInvH, (float)(kTgN - 1));
    const int i = min((int)t, kTgN - 2);
    const float f = t - (float)i;
    const float2 a = o.tg[i], b = o.tg[i + 1];
    fm = __builtin_fmaf(f, b.x - a.x, a.x);
    fs = __builtin_amdgcn_exp2f(__builtin_fmaf(f, b.y - a.y, a.y));
  }
  return fmaxf(m * __builtin_fmaf(fs, z1, fm), 0.0f);
}

// Broadie and Kaya's exact step (FP64; the FP32 state widened and rounded back).
__device__ __noinline__ void bk_transition(const DevOpt& o, float& x, float& v, const Draw& d) {
  const double vu = (double)v;
  const double vt = bk::variance(vu, o.bk_kappa, o.bk_theta, o.bk_xi, o.bk_dt, (double)d.u);
  const double iv = bk::integrated_variance(vu, vt, o.bk_kappa, o.bk_theta, o.bk_xi, o.bk_dt, (double)d.u2);
  const bool noisy = o.bk_xi > 0.0;
  const double wv = noisy ? (vt - vu - o.bk_kappa * o.bk_theta * o.bk_dt + o.bk_kappa * iv) / o.bk_xi : 0.0;
  const double rh = noisy ? o.bk_rho : 0.0;
  const double xn = (double)x + o.bk_r * o.bk_dt - 0.5 * iv + rh * wv + sqrt((1.0 - rh * rh) * iv) * (double)d.z2;
  x = (float)xn;
  v = (float)vt;
}

template <int SCHEME>
__device__ __forceinline__ void transition(const DevOpt& o, float& x, float& v, const Draw& d) {
  if constexpr (SCHEME == 0) {
    const float V = qe_variance(o, v, d.z1, d.u);
    x += qe_logprice_inc(o, v, V, d.z2);
    v = V;
  } else if constexpr (SCHEME == 4) {
    bk_transition(o, x, v, d);
  } else if constexpr (SCHEME == 3) {
    // truncated Gaussian variance, QE's log-price step
    const float V = tg_variance(o, v, d.z1);
    x += qe_logprice_inc(o, v, V, d.z2);
    v = V;
  } else if constexpr (SCHEME == 2) {
    // martingale-corrected QE: r dt + K0* in place of C0 = r dt + K0
    float g;
    bool ok;
    const float V = qe_variance_mgf(o, v, d.z1, d.u, g, ok);
    const float c0 = ok ? o.rdt - __builtin_fmaf(o.K13, v, g) : o.C0;
    const float w = __builtin_fmaf(o.K3, v, o.K4 * V);
    const float inc = __builtin_fmaf(o.K2, V, __builtin_fmaf(o.K1, v, c0));
    x += __builtin_fmaf(fsqrt(w), d.z2, inc);
    v = V;
  } else {
    fte_step(o, x, v, d.z1, d.z2);
  }
}

__device__ __forceinline__ bool is_call(int payoff) { return payoff == 0 || payoff == 3; }

// Intrinsic value h(S) of the option's call/put kind.
__device__ __forceinline__ float intrinsic(const DevOpt& o, float S) {
  const float h = is_call(o.payoff) ? S - o.K : o.K - S;
  return fmaxf(h, 0.0f);
}

// AssetPathExponential: S = S0 exp(x) (v_exp_f32 is exp2).
__device__ __forceinline__ float asset(const DevOpt& o, float x) {
  return o.S0 * __builtin_amdgcn_exp2f(x * 1.44269504088896340736f);
}

// ---------------------------------------------------------------------------------------------
// Compensated (Kahan) FP32 sum.
// ---------------------------------------------------------------------------------------------
struct Kahan {
  float s = 0.0f, c = 0.0f;
  __device__ __forceinline__ void add(float x) {
    const float y = x - c;
    const float t = s + y;
    c = (t - s) - y;
    s = t;
  }
  __device__ __forceinline__ double value() const { return (double)s - (double)c; }
};

// ---------------------------------------------------------------------------------------------
// Reductions.  Fixed butterfly order, so results are bitwise reproducible for a launch shape.
// ---------------------------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double x) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, kWave);
  return x;
}

// Wave64 sum of a float by DPP lane exchanges inside the VALU: two quad permutes, the
// half-row and row mirrors (every lane of a 16-lane row then holds the row sum), and the
// two row broadcasts (lane 63 then holds the wave sum), read back to all lanes.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ float dpp_term(float x) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, ROW_MASK, 0xF, false));
}

__device__ __forceinline__ float wave_sum(float x) {
  x += dpp_term<0xB1, 0xF>(x);   // quad_perm [1,0,3,2]
  x += dpp_term<0x4E, 0xF>(x);   // quad_perm [2,3,0,1]
  x += dpp_term<0x141, 0xF>(x);  // row_half_mirror
  x += dpp_term<0x140, 0xF>(x);  // row_mirror
  x += dpp_term<0x142, 0xA>(x);  // row_bcast:15 into rows 1 and 3
  x += dpp_term<0x143, 0xC>(x);  // row_bcast:31 into rows 2 and 3
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), 63));
}

// wave_sum of NV values at once, each DPP step applied to all of them before the next (the same
// operations per value, so the same bits; the independent chains overlap).
template <int NV>
__device__ __forceinline__ void wave_sum_n(float (&x)[NV]) {
#pragma unroll
  for (int a = 0; a < NV; ++a) x[a] += dpp_term<0xB1, 0xF>(x[a]);
#pragma unroll
  for (int a = 0; a < NV; ++a) x[a] += dpp_term<0x4E, 0xF>(x[a]);
#pragma unroll
  for (int a = 0; a < NV; ++a) x[a] += dpp_term<0x141, 0xF>(x[a]);
#pragma unroll
  for (int a = 0; a < NV; ++a) x[a] += dpp_term<0x140, 0xF>(x[a]);
#pragma unroll
  for (int a = 0; a < NV; ++a) x[a] += dpp_term<0x142, 0xA>(x[a]);
#pragma unroll
  for (int a = 0; a < NV; ++a) x[a] += dpp_term<0x143, 0xC>(x[a]);
#pragma unroll
  for (int a = 0; a < NV; ++a) x[a] = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x[a]), 63));
}

// Sums NV values per thread over the block; the result is valid in thread 0.
// `scratch` holds NV * (BLOCK / 64) elements of T.  Waves reduce in registers; the per-wave
// partials are then folded by wave 0, one partial per lane (float: a DPP sum; double: in
// wave order by thread 0).  The order is fixed, so results are reproducible.
template <int BLOCK, int NV, typename T>
__device__ __forceinline__ void block_sum(T (&vals)[NV], T* scratch) {
  constexpr int W = BLOCK / kWave;
  const int lane = threadIdx.x & (kWave - 1);
  const int wid = threadIdx.x / kWave;
#pragma unroll
  for (int i = 0; i < NV; ++i) vals[i] = wave_sum(vals[i]);
  if (W == 1) return;
  if (lane == 0) {
#pragma unroll
    for (int i = 0; i < NV; ++i) scratch[i * W + wid] = vals[i];
  }
  __syncthreads();
  if constexpr (sizeof(T) == 4) {
    if (wid == 0) {
#pragma unroll
      for (int i = 0; i < NV; ++i) vals[i] = wave_sum(lane < W ? scratch[i * W + lane] : T(0));
    }
  } else {
    if (threadIdx.x == 0) {
#pragma unroll
      for (int i = 0; i < NV; ++i) {
        T s = scratch[i * W];
        for (int w = 1; w < W; ++w) s += scratch[i * W + w];
        vals[i] = s;
      }
    }
  }
  __syncthreads();
}

}  // namespace simr
