// simr_api.hip -- host runtime and C ABI of the Heston Monte Carlo / Longstaff-Schwartz library.
//
// Responsibilities: argument validation before any launch; FP64 precomputation of the per-option
// step constants (rounded once to FP32) and of their derivatives for the adjoint chain rule;
// carving the caller's workspace; the tile autotuner; hipGraph capture and replay of the batch
// launch; FP64 finishing of prices, standard errors and Greeks on the host.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/simr.h"
#include "simr_kernels.hpp"

using namespace simr;

namespace {

thread_local std::string g_err;

simr_status fail(simr_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return s;
}

// Host-side fault injection (a test of the library's error paths; no kernel is affected).  A
// context may be armed to make its nth HIP call of one kind report a failure: allocations
// (hipMalloc, hipHostMalloc, hipEventCreate) and launches (kernels, graph launches) are then not
// made; copies and synchronisations are made and then reported as failed, so no work of the
// call is left in flight behind the error.  The plan of the context in use is reached through
// a thread-local pointer set for the duration of each call.
enum FaultKind { kFaultNone = 0, kFaultAlloc = 1, kFaultLaunch = 2, kFaultSync = 3, kFaultCreate = 4 };

struct FaultPlan {
  int kind = kFaultNone;
  int64_t countdown = 0;
  int64_t fired = 0;
};

thread_local FaultPlan* g_fault = nullptr;

const char* fault_name(int k) {
  return k == kFaultAlloc ? "alloc" : k == kFaultLaunch ? "launch" : k == kFaultSync ? "sync" : "create";
}

int hip_call_kind(const char* text) {
  if (std::strstr(text, "Malloc") || std::strstr(text, "EventCreate")) return kFaultAlloc;
  if (std::strncmp(text, "launch_", 7) == 0 || std::strstr(text, "GraphLaunch")) return kFaultLaunch;
  if (std::strstr(text, "Synchronize") || std::strstr(text, "Memcpy")) return kFaultSync;
  return kFaultNone;
}

// The kind of fault to report for this call (0: none).
int fault_check(const char* text) {
  FaultPlan* f = g_fault;
  if (!f || f->kind == kFaultNone || hip_call_kind(text) != f->kind) return kFaultNone;
  if (--f->countdown > 0) return kFaultNone;
  const int k = f->kind;
  f->kind = kFaultNone;
  ++f->fired;
  return k;
}

// "kind" or "kind:n" (n >= 1, default 1) into a plan.
bool parse_fault(const char* text, FaultPlan* plan) {
  static const char* names[] = {"alloc", "launch", "sync", "create"};
  for (int k = 0; k < 4; ++k) {
    const size_t n = std::strlen(names[k]);
    if (std::strncmp(text, names[k], n) != 0) continue;
    long long nth = 1;
    if (text[n] == ':') {
      char* end = nullptr;
      nth = std::strtoll(text + n + 1, &end, 10);
      if (end == text + n + 1 || *end != '\0' || nth < 1) return false;
    } else if (text[n] != '\0') {
      return false;
    }
    plan->kind = k + 1;
    plan->countdown = nth;
    return true;
  }
  return false;
}

#define SIMR_HIP(call)                                                                          \
  do {                                                                                          \
    const int fk_ = g_fault ? fault_check(#call) : 0;                                           \
    if (fk_ == kFaultAlloc || fk_ == kFaultLaunch)                                              \
      return fail(SIMR_EHIP, "injected %s failure: %s not made", fault_name(fk_), #call);       \
    hipError_t e_ = (call);                                                                     \
    if (fk_ == kFaultSync) return fail(SIMR_EHIP, "injected sync failure: %s", #call);          \
    if (e_ != hipSuccess) return fail(SIMR_EHIP, "%s: %s (%s:%d)", #call, hipGetErrorString(e_), \
                                      __FILE__, __LINE__);                                     \
  } while (0)

constexpr size_t kAlign = 256;
constexpr int kMaxSteps = 1 << 16;
constexpr int64_t kMaxPaths = (int64_t)1 << 30;

// Bump allocator over the caller's workspace; with base == nullptr it only measures.
struct Carve {
  char* base;
  size_t off = 0;
  explicit Carve(void* b) : base((char*)b) {}
  template <class T>
  T* take(size_t n) {
    off = (off + kAlign - 1) / kAlign * kAlign;
    T* p = base ? (T*)(base + off) : nullptr;
    off += std::max<size_t>(n, 1) * sizeof(T);
    return p;
  }
};

}  // namespace

// ---------------------------------------------------------------------------------------------
// Static device scratch of the allocation-free entry point (simr_price_noalloc): one array per
// device, in the device code object of this file, shared by every such call on that device and
// holding the last call's contents.  Host code never names it: simr_create takes its device
// address with hipGetSymbolAddress and every use goes through that address.
//   [0, 512)      the option record (DevOpt)
//   [512, 524)    the queue order {0} and unit prefix {0, tiles}
//   [1024, 1088)  the queue counter (16 words, cleared by a kernel before every launch)
//   [1280, 1296)  the result sums {sum X, sum X^2}
//   [2048, ...)   {sum X, sum X^2} per path tile, kScratchTiles tiles
// ---------------------------------------------------------------------------------------------
constexpr int64_t kScratchTiles = 131072;
constexpr size_t kScratchRecord = 512 + 3 * sizeof(int32_t);
constexpr size_t kScratchCounter = 1024;
constexpr size_t kScratchResult = 1280;
constexpr size_t kScratchPartials = 2048;
constexpr size_t kScratchBytes = kScratchPartials + 2 * sizeof(double) * (size_t)kScratchTiles;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

struct GraphEntry {
  hipGraphExec_t exec = nullptr;
};

struct ProfPair {
  int group;
  hipEvent_t a, b;
};

struct simr_ctx {
  int device = 0;
  bool prof_on = false;
  uint32_t prof_mask = (1u << SIMR_PROF_GROUPS) - 1;  // groups recorded while profiling
  std::vector<ProfPair> prof_pending;
  std::vector<hipEvent_t> prof_pool;
  double prof_ms[SIMR_PROF_GROUPS] = {};
  int64_t prof_n[SIMR_PROF_GROUPS] = {};
  int num_cus = 0;
  std::string arch;
  int lsm_grid_max = 64;       // largest cooperative grid of the backward induction
  int lsm_block = 0;           // its block size: 0 chosen per launch, or fixed at 1024 or 256
  bool lsm_per_date = false;   // force one launch per date instead of the cooperative kernel
  bool lsm_fail_test = false;  // mark the exchange as failed before each cooperative induction
  int tile_block[5] = {0, 0, 0, 0, 0};  // per scheme: 0 = not chosen yet
  int tile_ppl[5] = {0, 0, 0, 0, 0};
  float2* tg = nullptr;              // truncated Gaussian table (device), built by simr_create
  char* scratch = nullptr;           // device address of this device's static scratch array
  double* noalloc_sums = nullptr;    // pinned host landing of simr_price_noalloc's result sums
  int64_t graph_captures = 0;        // batch graphs captured / launched (capture or replay)
  int64_t graph_launches = 0;
  void* pinned = nullptr;
  size_t pinned_bytes = 0;
  FaultPlan fault;
  std::map<std::tuple<uintptr_t, uintptr_t, int, int, int, int, int, int, uintptr_t>, GraphEntry> graphs;
};

namespace {

// Records HIP events around a group of launches on the call's stream when profiling is on.
struct Prof {
  simr_ctx* c;
  int group;
  hipStream_t s;
  hipEvent_t a = nullptr;
  hipEvent_t take() {
    if (!c->prof_pool.empty()) {
      hipEvent_t e = c->prof_pool.back();
      c->prof_pool.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
  }
  Prof(simr_ctx* c_, int g, hipStream_t s_) : c(c_), group(g), s(s_) {
    if (c->prof_on && ((c->prof_mask >> group) & 1u) && (a = take())) (void)hipEventRecord(a, s);
  }
  ~Prof() {
    if (!a) return;
    hipEvent_t b = take();
    if (!b) return;
    (void)hipEventRecord(b, s);
    c->prof_pending.push_back(ProfPair{group, a, b});
  }
};

// Makes the context's device current for a call (and its fault plan the one in use).
struct DeviceGuard {
  int old = -1;
  FaultPlan* old_fault = nullptr;
  explicit DeviceGuard(int dev) { enter(dev); }
  explicit DeviceGuard(simr_ctx* c) {
    enter(c->device);
    old_fault = g_fault;
    g_fault = &c->fault;
  }
  void enter(int dev) {
    old_fault = g_fault;
    if (hipGetDevice(&old) != hipSuccess) old = -1;
    if (old != dev) (void)hipSetDevice(dev);
  }
  ~DeviceGuard() {
    g_fault = old_fault;
    if (old >= 0) (void)hipSetDevice(old);
  }
};

bool finite(double x) { return std::isfinite(x); }

simr_status validate_params(const simr_params* prm, int* scheme, int* ck) {
  if (!prm) return fail(SIMR_EINVAL, "params is NULL");
  if (prm->scheme != SIMR_SCHEME_QE && prm->scheme != SIMR_SCHEME_FTE && prm->scheme != SIMR_SCHEME_QE_M &&
      prm->scheme != SIMR_SCHEME_TG && prm->scheme != SIMR_SCHEME_BK)
    return fail(SIMR_EINVAL, "unknown scheme %d", prm->scheme);
  int c = prm->checkpoint_every == 0 ? 16 : prm->checkpoint_every;
  if (c != 8 && c != 16 && c != 32) return fail(SIMR_EINVAL, "checkpoint_every must be 0, 8, 16 or 32 (got %d)", c);
  if (prm->flags != 0 || prm->reserved != 0) return fail(SIMR_EINVAL, "params.flags and params.reserved must be 0");
  *scheme = prm->scheme;
  *ck = c;
  return SIMR_OK;
}

simr_status validate_option(const simr_option* o, int64_t i) {
  if (!o) return fail(SIMR_EINVAL, "option pointer is NULL");
  const double v[] = {o->S0, o->K, o->T, o->r, o->kappa, o->theta, o->xi, o->rho, o->v0};
  for (double x : v)
    if (!finite(x)) return fail(SIMR_EINVAL, "option %lld: non-finite parameter", (long long)i);
  if (!(o->S0 > 0) || !(o->K > 0) || !(o->T > 0))
    return fail(SIMR_EINVAL, "option %lld: S0, K and T must be > 0", (long long)i);
  if (!(o->kappa > 0) || !(o->theta > 0)) return fail(SIMR_EINVAL, "option %lld: kappa and theta must be > 0", (long long)i);
  if (o->v0 < 0 || o->xi < 0) return fail(SIMR_EINVAL, "option %lld: v0 and xi must be >= 0", (long long)i);
  if (!(std::fabs(o->rho) <= 1.0)) return fail(SIMR_EINVAL, "option %lld: |rho| must be <= 1", (long long)i);
  if (o->payoff < SIMR_EURO_CALL || o->payoff > SIMR_AMER_CALL)
    return fail(SIMR_EINVAL, "option %lld: unknown payoff %d", (long long)i, o->payoff);
  if (o->steps < 1 || o->steps > kMaxSteps)
    return fail(SIMR_EINVAL, "option %lld: steps must be in [1, %d]", (long long)i, kMaxSteps);
  if (o->paths < 2 || o->paths > kMaxPaths)
    return fail(SIMR_EINVAL, "option %lld: paths must be in [2, 2^30]", (long long)i);
  if (o->reserved != 0) return fail(SIMR_EINVAL, "option %lld: reserved must be 0", (long long)i);
  return SIMR_OK;
}

bool american(const simr_option& o) { return o.payoff == SIMR_AMER_PUT || o.payoff == SIMR_AMER_CALL; }

// Step constants of one option, FP64 -> FP32, plus their derivatives for the adjoint.
DevOpt make_devopt(const simr_option& o) {
  DevOpt d;
  std::memset(&d, 0, sizeof d);
  const double dt = o.T / o.steps;
  const double E = std::exp(-o.kappa * dt);
  const double omE = -std::expm1(-o.kappa * dt);
  const double xi2 = o.xi * o.xi;
  const double A1 = xi2 * E * omE / o.kappa;
  const double A2 = o.theta * xi2 * omE * omE / (2.0 * o.kappa);
  const bool sv = o.xi > 0.0;  // with xi = 0 the variance is deterministic and rho drops out
  const double rho = sv ? o.rho : 0.0;
  const double rox = sv ? rho / o.xi : 0.0;
  const double K0 = sv ? -rho * o.kappa * o.theta * dt / o.xi : 0.0;
  const double K1 = 0.5 * dt * (o.kappa * rox - 0.5) - rox;
  const double K2 = 0.5 * dt * (o.kappa * rox - 0.5) + rox;
  const double K3 = 0.5 * dt * (1.0 - rho * rho);
  d.E = (float)E;
  d.A1 = (float)A1;
  d.A2 = (float)A2;
  d.theta = (float)o.theta;
  d.C0 = (float)(o.r * dt + K0);
  d.K1 = (float)K1;
  d.K2 = (float)K2;
  d.K3 = (float)K3;
  d.K4 = (float)K3;
  d.Amg = (float)(K2 + 0.5 * K3);  // K4 = K3 (gamma1 = gamma2)
  d.K13 = (float)(K1 + 0.5 * K3);
  d.kdt = (float)(o.kappa * dt);
  d.kthdt = (float)(o.kappa * o.theta * dt);
  d.xisdt = (float)(o.xi * std::sqrt(dt));
  d.sdt = (float)std::sqrt(dt);
  d.hdt = (float)(0.5 * dt);
  d.rdt = (float)(o.r * dt);
  d.rho = (float)o.rho;
  d.srho = (float)std::sqrt(std::max(0.0, 1.0 - o.rho * o.rho));
  d.S0 = (float)o.S0;
  d.K = (float)o.K;
  d.disc = (float)std::exp(-o.r * o.T);
  d.v0 = (float)o.v0;
  d.invK = (float)(1.0 / o.K);
  d.invTheta = (float)(1.0 / o.theta);
  // derivatives of the step constants with respect to (theta, r, kappa, xi, rho)
  const double dE_dk = -dt * E;
  d.dE_dk = (float)dE_dk;
  d.dA1_dk = (float)(xi2 * dE_dk * (1.0 - 2.0 * E) / o.kappa - A1 / o.kappa);
  d.dA1_dxi = (float)(2.0 * o.xi * E * omE / o.kappa);
  d.dA2_dth = (float)(xi2 * omE * omE / (2.0 * o.kappa));
  d.dA2_dk = (float)(-o.theta * xi2 * omE * dE_dk / o.kappa - A2 / o.kappa);
  d.dA2_dxi = (float)(o.theta * o.xi * omE * omE / o.kappa);
  d.dC0_dr = (float)dt;
  if (sv) {
    const double ix = 1.0 / o.xi;
    d.dC0_dth = (float)(-rho * o.kappa * dt * ix);
    d.dC0_dk = (float)(-rho * o.theta * dt * ix);
    d.dC0_dxi = (float)(rho * o.kappa * o.theta * dt * ix * ix);
    d.dC0_drho = (float)(-o.kappa * o.theta * dt * ix);
    d.dK1_dk = (float)(0.5 * dt * rho * ix);
    d.dK1_dxi = (float)(-0.5 * dt * o.kappa * rho * ix * ix + rho * ix * ix);
    d.dK1_drho = (float)(0.5 * dt * o.kappa * ix - ix);
    d.dK2_dk = (float)(0.5 * dt * rho * ix);
    d.dK2_dxi = (float)(-0.5 * dt * o.kappa * rho * ix * ix - rho * ix * ix);
    d.dK2_drho = (float)(0.5 * dt * o.kappa * ix + ix);
    d.dK3_drho = (float)(-dt * rho);
    d.dK4_drho = (float)(-dt * rho);
  }
  // maturity: every constant depends on T through dt = T / N (d dt / dT = 1 / N)
  {
    const double iN = 1.0 / o.steps;
    const double dEdT = -o.kappa * E * iN;
    d.dE_dT = (float)dEdT;
    d.dA1_dT = (float)(xi2 * (1.0 - 2.0 * E) / o.kappa * dEdT);
    d.dA2_dT = (float)(-o.theta * xi2 * omE / o.kappa * dEdT);
    d.dC0_dT = (float)((o.r + (sv ? -rho * o.kappa * o.theta / o.xi : 0.0)) * iN);
    d.dK1_dT = (float)(0.5 * (o.kappa * rox - 0.5) * iN);
    d.dK2_dT = (float)(0.5 * (o.kappa * rox - 0.5) * iN);
    d.dK3_dT = (float)(0.5 * (1.0 - rho * rho) * iN);
    d.rN = (float)(o.r * iN);
    const double isdt = 1.0 / std::sqrt(dt);
    d.fdT_rdt = (float)(o.r * iN);
    d.fdT_hdt = (float)(0.5 * iN);
    d.fdT_sdt = (float)(0.5 * isdt * iN);
    d.fdT_kdt = (float)(o.kappa * iN);
    d.fdT_kthdt = (float)(o.kappa * o.theta * iN);
    d.fdT_xisdt = (float)(0.5 * o.xi * isdt * iN);
  }
  d.dt = (float)dt;
  d.payoff = o.payoff;
  d.steps = o.steps;
  d.paths = (int32_t)o.paths;
  d.bk_kappa = o.kappa;
  d.bk_theta = o.theta;
  d.bk_xi = o.xi;
  d.bk_rho = o.rho;
  d.bk_r = o.r;
  d.bk_dt = o.T / o.steps;
  d.stream = o.stream_id;
  d.seed_lo = (uint32_t)(o.seed & 0xffffffffu);
  d.seed_hi = (uint32_t)(o.seed >> 32);
  return d;
}

static_assert(sizeof(DevOpt) <= 512, "the autotuner stages one DevOpt in the first 512 bytes");

// Moment matching of the truncated Gaussian scheme: with A = r Phi(r) + phi(r) (= E[Y] / sigma)
// and B = (r^2 + 1) Phi(r) + r phi(r) (= E[Y^2] / sigma^2) for Y = max(mu + sigma Z, 0), r = mu /
// sigma solves log B - 2 log A = log(1 + psi); dA/dr = Phi, dB/dr = 2 A.  Safeguarded Newton.
void tg_parts(double r, double* A, double* B, double* P) {
  *P = 0.5 * std::erfc(-r / std::sqrt(2.0));
  const double f = std::exp(-0.5 * r * r) / std::sqrt(2.0 * M_PI);
  *A = r * *P + f;
  *B = (r * r + 1.0) * *P + r * f;
}

double tg_solve_r(double psi) {
  const double target = std::log1p(psi);
  double lo = -64.0, hi = 1.0 / std::sqrt(psi) + 1.0;  // F(lo) > 0 > F(hi)
  double r = psi < 1.0 ? 1.0 / std::sqrt(psi) : 0.0;
  for (int it = 0; it < 200; ++it) {
    double A, B, P;
    tg_parts(r, &A, &B, &P);
    const double F = std::log(B) - 2.0 * std::log(A) - target;
    if (F > 0.0)
      lo = r;
    else
      hi = r;
    const double dF = 2.0 * A / B - 2.0 * P / A;
    double rn = r - F / dF;
    if (!(rn > lo && rn < hi)) rn = 0.5 * (lo + hi);
    if (std::fabs(rn - r) <= 1e-15 * std::max(1.0, std::fabs(r))) return rn;
    r = rn;
  }
  return r;
}

// The truncated Gaussian table: kTgN nodes uniform in l = log2(psi), first (mu / m, log2(sigma / m)),
// then their derivatives in l (for the adjoint), exact in FP64 at the nodes.  With
// mu / m = r / A(r), sigma / m = 1 / A(r), A' = Phi, A - r Phi = phi and
// dr/dpsi = A^3 / (2 (A^2 - B Phi)) (implicit differentiation of B / A^2 = 1 + psi), and
// dpsi/dl = psi ln 2: d(mu / m)/dl = phi / A^2 r' psi ln 2, d log2(sigma / m)/dl = -Phi / A r' psi.
simr_status build_tg_table(simr_ctx* c) {
  if (c->tg) return SIMR_OK;
  std::vector<float2> t(2 * (size_t)kTgN);
  for (int i = 0; i < kTgN; ++i) {
    const double lp = kTgLo + (double)i * (double)(kTgHi - kTgLo) / (kTgN - 1);
    const double psi = std::exp2(lp);
    const double r = tg_solve_r(psi);
    double A, B, P;
    tg_parts(r, &A, &B, &P);
    t[i].x = (float)(r / A);          // mu / m
    t[i].y = (float)(-std::log2(A));  // log2(sigma / m)
    const double dr = A * A * A / (2.0 * (A * A - B * P));
    const double phi = A - r * P;
    t[kTgN + i].x = (float)(phi / (A * A) * dr * psi * M_LN2);
    t[kTgN + i].y = (float)(-P / A * dr * psi);
  }
  float2* d = nullptr;
  SIMR_HIP(hipMalloc(&d, sizeof(float2) * t.size()));
  const hipError_t e = hipMemcpy(d, t.data(), sizeof(float2) * t.size(), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    (void)hipFree(d);
    return fail(SIMR_EHIP, "hipMemcpy: %s", hipGetErrorString(e));
  }
  c->tg = d;
  return SIMR_OK;
}

// The device constants of an option under `scheme` (the truncated Gaussian table attached; the
// table is built once by simr_create, so no call after it allocates device memory).
simr_status devopt_for(simr_ctx* c, int scheme, const simr_option& o, DevOpt* d) {
  *d = make_devopt(o);
  d->tg = nullptr;
  if (scheme == SIMR_SCHEME_TG) {
    if (!c->tg) return fail(SIMR_EINVAL, "internal: the truncated Gaussian table is missing");
    d->tg = c->tg;
  }
  return SIMR_OK;
}

double intrinsic_host(const simr_option& o, double S) {
  const double h = (o.payoff == SIMR_EURO_CALL || o.payoff == SIMR_AMER_CALL) ? S - o.K : o.K - S;
  return h > 0 ? h : 0.0;
}

void mean_se(double s1, double s2, int64_t P, double* mean, double* se) {
  const double m = s1 / (double)P;
  double var = (s2 - s1 * s1 / (double)P) / (double)(P - 1);
  if (var < 0) var = 0;
  *mean = m;
  *se = std::sqrt(var / (double)P);
}

simr_status ensure_pinned(simr_ctx* c, size_t bytes) {
  if (c->pinned_bytes >= bytes) return SIMR_OK;
  if (c->pinned) (void)hipHostFree(c->pinned);
  c->pinned = nullptr;
  c->pinned_bytes = 0;
  size_t want = std::max<size_t>(bytes, 1 << 16);
  SIMR_HIP(hipHostMalloc(&c->pinned, want, hipHostMallocDefault));
  c->pinned_bytes = want;
  // graphs hold the old staging address
  for (auto& kv : c->graphs) (void)hipGraphExecDestroy(kv.second.exec);
  c->graphs.clear();
  return SIMR_OK;
}

// ---------------------------------------------------------------------------------------------
// Workspace layouts.
// ---------------------------------------------------------------------------------------------
struct LsmBufs {
  float* gram;   // Gram sums of every (date, chunk)
  double* fac;   // factor record of every date
  float *xs, *vs, *hcash;
  int32_t* tau;
  LsmState st;   // per-date launches; st.flags also collects the factor flags
  unsigned long long* xchg;  // exchange words of the cooperative induction
  double* partials;  // 2 per block
  int nblk;
};

// uint32 words per option that are zero before an induction: ticket, flags, ... (16), exchange
constexpr int64_t kOptZeroWords = 16 + 2 * (int64_t)kLsmXchgWords;

LsmBufs carve_lsm(Carve& cv, int64_t P, int N, uint32_t* words) {
  LsmBufs b;
  b.nblk = (int)((P + kLsmBlock - 1) / kLsmBlock);
  b.xs = cv.take<float>((size_t)P * N);
  b.vs = cv.take<float>((size_t)P * N);
  b.hcash = cv.take<float>(P);
  b.tau = cv.take<int32_t>(P);
  b.st.gpart = cv.take<float>((size_t)b.nblk * 32 * 2);  // per-date launches use one half
  b.st.ticket = words;
  b.st.flags = words ? (int32_t*)(words + 1) : nullptr;
  b.xchg = words ? (unsigned long long*)(words + 16) : nullptr;
  b.st.beta32 = cv.take<float>((size_t)(N + 1) * 8);
  b.st.beta64 = cv.take<double>((size_t)(N + 1) * 6);
  b.gram = cv.take<float>((size_t)(N + 1) * lsm_gram_chunks(P) * kLsmGramRow);
  b.fac = cv.take<double>((size_t)(N + 1) * kLsmFacRec);
  b.partials = cv.take<double>((size_t)b.nblk * 2);
  return b;
}

// The American options of one pass: every option keeps its own spill, factors and exchange
// words; the words that must start at zero are contiguous, so one launch clears them.
struct AmerGroup {
  std::vector<int64_t> idx;  // indices into the caller's option array
  std::vector<LsmBufs> b;
  uint32_t* zero;            // [option][kOptZeroWords], then 16 words of the group (status)
  int64_t zero_words;
  int32_t* status;
  LsmTask* tasks;            // one per option
  double* results;           // 2 doubles per option, then int32 flags per option and the status
};

AmerGroup carve_amer_group(Carve& cv, const simr_option* opts, const std::vector<int64_t>& idx) {
  AmerGroup g;
  g.idx = idx;
  const int64_t n = (int64_t)idx.size();
  g.zero_words = n * kOptZeroWords + 16;
  g.zero = cv.take<uint32_t>((size_t)g.zero_words);
  g.status = g.zero ? (int32_t*)(g.zero + n * kOptZeroWords) : nullptr;
  g.tasks = cv.take<LsmTask>((size_t)n);
  g.results = cv.take<double>((size_t)(3 * n + 1));
  for (int64_t k = 0; k < n; ++k)
    g.b.push_back(carve_lsm(cv, opts[idx[k]].paths, opts[idx[k]].steps, g.zero ? g.zero + k * kOptZeroWords : nullptr));
  return g;
}

size_t amer_group_bytes(const simr_option* opts, const std::vector<int64_t>& idx) {
  Carve cv(nullptr);
  carve_amer_group(cv, opts, idx);
  return cv.off;
}

// The American options of a batch in passes of consecutive options (caller's order) whose
// buffers fit kAmerPassBytes together, or one option alone if it needs more.
constexpr size_t kAmerPassBytes = (size_t)8 << 30;

std::vector<std::vector<int64_t>> amer_passes(const simr_option* opts, const std::vector<int64_t>& amer) {
  std::vector<std::vector<int64_t>> out;
  std::vector<int64_t> cur;
  size_t bytes = 0;
  for (int64_t i : amer) {
    const size_t one = amer_group_bytes(opts, {i});
    if (!cur.empty() && bytes + one > kAmerPassBytes) {
      out.push_back(cur);
      cur.clear();
      bytes = 0;
    }
    cur.push_back(i);
    bytes += one;
  }
  if (!cur.empty()) out.push_back(cur);
  return out;
}

struct BatchBufs {
  char* upload;        // [opts | order | uprefix], mirrored in pinned staging
  size_t upload_bytes;
  DevOpt* opts;
  int32_t* order;
  int32_t* uprefix;
  uint32_t* counter;
  double* partials;
  double* results;     // 2 per option
  size_t off_order, off_uprefix;
};

BatchBufs carve_batch(Carve& cv, int64_t n, int64_t total_tiles) {
  BatchBufs b;
  const size_t so = sizeof(DevOpt) * (size_t)n;
  b.off_order = (so + kAlign - 1) / kAlign * kAlign;
  b.off_uprefix = b.off_order + ((sizeof(int32_t) * (size_t)n + kAlign - 1) / kAlign * kAlign);
  b.upload_bytes = b.off_uprefix + sizeof(int32_t) * (size_t)(n + 1);
  b.upload = cv.take<char>(b.upload_bytes);
  b.opts = (DevOpt*)b.upload;
  b.order = b.upload ? (int32_t*)(b.upload + b.off_order) : nullptr;
  b.uprefix = b.upload ? (int32_t*)(b.upload + b.off_uprefix) : nullptr;
  b.counter = cv.take<uint32_t>(16);
  b.partials = cv.take<double>((size_t)total_tiles * 2);
  b.results = cv.take<double>((size_t)n * 2);
  return b;
}

// Calibration area of the autotuner (inside every batch workspace).
constexpr int kTuneTiles = 8192;
struct TuneBufs {
  char* upload;
  uint32_t* counter;
  double* partials;
};
TuneBufs carve_tune(Carve& cv) {
  TuneBufs t;
  t.upload = cv.take<char>(1024);
  t.counter = cv.take<uint32_t>(16);
  t.partials = cv.take<double>((size_t)kTuneTiles * 2);
  return t;
}

constexpr int kGreekResultDoubles = 2 + 2 * SIMR_NUM_GREEKS_EXT;  // price sums, Greek sums, squares

struct GreekBufs {
  float *ck, *xN;
  double *partials, *gpart, *result;
  int nblk;      // blocks of the checkpointing forward pass (2 partials each)
  int nblk_adj;  // rows of 14 partials room is carved for: blocks of the smallest adjoint block
};

GreekBufs carve_greeks_euro(Carve& cv, int64_t P, int N, int CK) {
  GreekBufs g;
  g.nblk = (int)((P + kCkBlock - 1) / kCkBlock);
  g.nblk_adj = (int)((P + kAdjMinBlock - 1) / kAdjMinBlock);
  const int nseg = (N + CK - 1) / CK;
  g.ck = cv.take<float>((size_t)std::max(nseg - 1, 1) * P);
  g.xN = cv.take<float>(P);
  g.partials = cv.take<double>((size_t)g.nblk * 2);
  g.gpart = cv.take<double>((size_t)g.nblk_adj * 2 * SIMR_NUM_GREEKS_EXT);
  g.result = cv.take<double>(kGreekResultDoubles);
  return g;
}

struct BatchPlan {
  std::vector<int64_t> euro, amer;  // indices into the caller's array
  int64_t total_tiles = 0;
};

BatchPlan plan_batch(const simr_option* opts, int64_t n, int tile_paths) {
  BatchPlan pl;
  for (int64_t i = 0; i < n; ++i) {
    if (american(opts[i])) {
      pl.amer.push_back(i);
    } else {
      pl.euro.push_back(i);
      pl.total_tiles += (opts[i].paths + tile_paths - 1) / tile_paths;
    }
  }
  return pl;
}

size_t batch_bytes(const simr_option* opts, int64_t n, int tile_paths) {
  BatchPlan pl = plan_batch(opts, n, tile_paths);
  Carve cv(nullptr);
  carve_tune(cv);
  carve_batch(cv, (int64_t)pl.euro.size(), pl.total_tiles);
  size_t amer = 0;
  for (const auto& grp : amer_passes(opts, pl.amer)) amer = std::max(amer, amer_group_bytes(opts, grp));
  return cv.off + (amer ? amer + kAlign : 0);
}

// The largest tile any candidate uses, so the workspace fits whatever the tuner picks.
constexpr int kMaxTilePaths = 256 * 4;
constexpr int kMinTilePaths = 128;

// ---------------------------------------------------------------------------------------------
// Autotuner: times the batch kernel for each (block, paths per lane) candidate on a calibration
// workload (C1-like Heston option, 64 steps, enough tiles to fill the GPU several times) and
// keeps the fastest.  Optionally cached across processes in the file named by
// SIMR_AUTOTUNE_CACHE ("<arch> <CUs> <scheme> <block> <ppl>" lines).
// ---------------------------------------------------------------------------------------------
const int kCandidates[][2] = {{128, 1}, {128, 2}, {128, 4}, {256, 1}, {256, 2}, {256, 4}};

bool load_tune_cache(simr_ctx* c, int scheme) {
  const char* path = std::getenv("SIMR_AUTOTUNE_CACHE");
  if (!path) return false;
  FILE* f = std::fopen(path, "r");
  if (!f) return false;
  char arch[128];
  int cus, sch, blk, ppl;
  bool found = false;
  while (std::fscanf(f, "%127s %d %d %d %d", arch, &cus, &sch, &blk, &ppl) == 5) {
    if (c->arch == arch && cus == c->num_cus && sch == scheme) {
      for (auto& cand : kCandidates)
        if (cand[0] == blk && cand[1] == ppl) {
          c->tile_block[scheme] = blk;
          c->tile_ppl[scheme] = ppl;
          found = true;
        }
    }
  }
  std::fclose(f);
  return found;  // a corrupt or foreign cache falls back to tuning
}

void save_tune_cache(simr_ctx* c, int scheme) {
  const char* path = std::getenv("SIMR_AUTOTUNE_CACHE");
  if (!path) return;
  FILE* f = std::fopen(path, "a");
  if (!f) return;
  std::fprintf(f, "%s %d %d %d %d\n", c->arch.c_str(), c->num_cus, scheme, c->tile_block[scheme], c->tile_ppl[scheme]);
  std::fclose(f);
}

int grid_for(simr_ctx* c, int scheme, int block, int ppl, int64_t nunits) {
  int occ = batch_kernel_occupancy(scheme, block, ppl);
  if (occ < 1) occ = 1;
  int64_t g = (int64_t)c->num_cus * occ;
  return (int)std::max<int64_t>(1, std::min<int64_t>(g, nunits));
}

simr_status autotune(simr_ctx* c, int scheme, const TuneBufs& tb, hipStream_t s) {
  if (c->tile_block[scheme]) return SIMR_OK;
  if (scheme == SIMR_SCHEME_BK) {  // FP64-bound at ~1e6 operations per step: a fixed tile, no timing runs
    c->tile_block[scheme] = 256;
    c->tile_ppl[scheme] = 1;
    return SIMR_OK;
  }
  if (load_tune_cache(c, scheme)) return SIMR_OK;
  simr_option o;
  std::memset(&o, 0, sizeof o);
  o.S0 = 100; o.K = 100; o.T = 1; o.r = 0.02; o.kappa = 1.5; o.theta = 0.04; o.xi = 0.3; o.rho = -0.7; o.v0 = 0.04;
  o.payoff = SIMR_EURO_CALL;
  o.steps = 64;
  o.seed = 12345;
  hipEvent_t e0, e1;
  SIMR_HIP(hipEventCreate(&e0));
  SIMR_HIP(hipEventCreate(&e1));
  float best = 1e30f;
  int bb = 256, bp = 1;
  simr_status st = ensure_pinned(c, 1024);
  if (st != SIMR_OK) return st;
  for (auto& cand : kCandidates) {
    const int tile = cand[0] * cand[1];
    const int64_t tiles = std::min<int64_t>(kTuneTiles, (int64_t)c->num_cus * 8 * 1024 / tile);
    o.paths = tiles * tile;
    DevOpt d;
    if ((st = devopt_for(c, scheme, o, &d)) != SIMR_OK) return st;
    d.slot0 = 0;
    d.ntiles = (int32_t)tiles;
    char* up = (char*)c->pinned;
    std::memcpy(up, &d, sizeof d);
    int32_t* ord = (int32_t*)(up + 512);
    ord[0] = 0;
    ord[1] = 0;
    ord[2] = (int32_t)tiles;  // uprefix = {0, tiles}
    SIMR_HIP(hipMemcpyAsync(tb.upload, up, 1024, hipMemcpyHostToDevice, s));
    BatchLaunch L;
    L.opts = (const DevOpt*)tb.upload;
    L.order = (const int32_t*)(tb.upload + 512);
    L.uprefix = (const int32_t*)(tb.upload + 516);
    L.nopt = 1;
    L.nunits = (int32_t)tiles;
    L.counter = tb.counter;
    L.partials = tb.partials;
    L.block = cand[0];
    L.ppl = cand[1];
    L.grid = grid_for(c, scheme, cand[0], cand[1], tiles);
    float ms_min = 1e30f;
    for (int rep = 0; rep < 3; ++rep) {  // first repetition warms up
      SIMR_HIP(launch_reset_words(tb.counter, 16, s));
      SIMR_HIP(hipEventRecord(e0, s));
      SIMR_HIP(launch_batch_price(scheme, L, s));
      SIMR_HIP(hipEventRecord(e1, s));
      SIMR_HIP(hipEventSynchronize(e1));
      float ms = 0;
      SIMR_HIP(hipEventElapsedTime(&ms, e0, e1));
      if (rep > 0) ms_min = std::min(ms_min, ms);
    }
    const float per_path = ms_min / (float)o.paths;
    if (per_path < best) {
      best = per_path;
      bb = cand[0];
      bp = cand[1];
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  c->tile_block[scheme] = bb;
  c->tile_ppl[scheme] = bp;
  save_tune_cache(c, scheme);
  return SIMR_OK;
}

// ---------------------------------------------------------------------------------------------
// European batch: upload the option table, reset the queue, persistent launch, finalize,
// download -- captured once per shape into a hipGraph and replayed.
// ---------------------------------------------------------------------------------------------
simr_status run_euro_batch(simr_ctx* c, int scheme, const simr_option* opts, const std::vector<int64_t>& idx,
                           const BatchBufs& b, int64_t total_tiles, simr_result* out, hipStream_t s) {
  const int64_t m = (int64_t)idx.size();
  if (m == 0) return SIMR_OK;
  const int block = c->tile_block[scheme], ppl = c->tile_ppl[scheme];
  const int tile = block * ppl;
  // host tables: constants, order by descending cost, unit prefix sums
  const size_t res_off = (b.upload_bytes + kAlign - 1) / kAlign * kAlign;
  simr_status st = ensure_pinned(c, res_off + sizeof(double) * 2 * (size_t)m);
  if (st != SIMR_OK) return st;
  char* up = (char*)c->pinned;
  DevOpt* dopt = (DevOpt*)up;
  int32_t* order = (int32_t*)(up + b.off_order);
  int32_t* uprefix = (int32_t*)(up + b.off_uprefix);
  std::vector<int64_t> ntile(m);
  int32_t slot = 0;
  for (int64_t k = 0; k < m; ++k) {
    const simr_option& o = opts[idx[k]];
    if ((st = devopt_for(c, scheme, o, &dopt[k])) != SIMR_OK) return st;
    ntile[k] = (o.paths + tile - 1) / tile;
    dopt[k].slot0 = slot;
    dopt[k].ntiles = (int32_t)ntile[k];
    slot += (int32_t)ntile[k];
    order[k] = (int32_t)k;
  }
  std::stable_sort(order, order + m, [&](int32_t a, int32_t bq) {
    const double ca = (double)opts[idx[a]].steps * (double)opts[idx[a]].paths;
    const double cb = (double)opts[idx[bq]].steps * (double)opts[idx[bq]].paths;
    return ca > cb;
  });
  uprefix[0] = 0;
  for (int64_t k = 0; k < m; ++k) uprefix[k + 1] = uprefix[k] + (int32_t)ntile[order[k]];
  const int32_t nunits = uprefix[m];
  if ((int64_t)nunits != total_tiles) return fail(SIMR_EINVAL, "internal: unit count mismatch");
  double* res_host = (double*)(up + res_off);

  BatchLaunch L;
  L.opts = b.opts;
  L.order = b.order;
  L.uprefix = b.uprefix;
  L.nopt = (int32_t)m;
  L.nunits = nunits;
  L.counter = b.counter;
  L.partials = b.partials;
  L.block = block;
  L.ppl = ppl;
  L.grid = grid_for(c, scheme, block, ppl, nunits);

  auto enqueue = [&]() -> simr_status {
    SIMR_HIP(hipMemcpyAsync(b.upload, up, b.upload_bytes, hipMemcpyHostToDevice, s));
    SIMR_HIP(launch_reset_words(b.counter, 16, s));
    {
      Prof pf(c, SIMR_PROF_PRICE, s);
      SIMR_HIP(launch_batch_price(scheme, L, s));
    }
    SIMR_HIP(launch_finalize_rows(b.partials, 2, b.opts, (int)m, 0, b.results, s));
    SIMR_HIP(hipMemcpyAsync(res_host, b.results, sizeof(double) * 2 * (size_t)m, hipMemcpyDeviceToHost, s));
    return SIMR_OK;
  };

  if (s != nullptr && !c->prof_on) {
    auto key = std::make_tuple((uintptr_t)b.upload, (uintptr_t)c->pinned, (int)m, (int)nunits, block, ppl, scheme,
                               L.grid, (uintptr_t)s);
    auto it = c->graphs.find(key);
    if (it == c->graphs.end()) {
      hipGraph_t g = nullptr;
      SIMR_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeRelaxed));
      simr_status es = enqueue();
      hipError_t ce = hipStreamEndCapture(s, &g);
      if (es != SIMR_OK) { if (g) (void)hipGraphDestroy(g); return es; }
      if (ce != hipSuccess) return fail(SIMR_EHIP, "hipStreamEndCapture: %s", hipGetErrorString(ce));
      hipGraphExec_t ex = nullptr;
      hipError_t ie = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      if (ie != hipSuccess) return fail(SIMR_EHIP, "hipGraphInstantiate: %s", hipGetErrorString(ie));
      if (c->graphs.size() >= 16) {
        for (auto& kv : c->graphs) (void)hipGraphExecDestroy(kv.second.exec);
        c->graphs.clear();
      }
      it = c->graphs.emplace(key, GraphEntry{ex}).first;
      ++c->graph_captures;
    }
    SIMR_HIP(hipGraphLaunch(it->second.exec, s));
    ++c->graph_launches;
  } else {
    simr_status es = enqueue();
    if (es != SIMR_OK) return es;
  }
  SIMR_HIP(hipStreamSynchronize(s));
  for (int64_t k = 0; k < m; ++k) {
    simr_result r;
    std::memset(&r, 0, sizeof r);
    mean_se(res_host[2 * k], res_host[2 * k + 1], opts[idx[k]].paths, &r.price, &r.std_err);
    r.paths = opts[idx[k]].paths;
    out[idx[k]] = r;
  }
  return SIMR_OK;
}

// Pinned staging of one American pass: the task table, then the results read back (2 doubles
// per option, then int32 flags per option and the status).
size_t amer_task_bytes(int n) { return (sizeof(LsmTask) * (size_t)n + kAlign - 1) / kAlign * kAlign; }
size_t amer_result_bytes(int n) { return sizeof(double) * 2 * (size_t)n + sizeof(int32_t) * (size_t)(n + 1); }
size_t amer_pinned_bytes(int n) { return amer_task_bytes(n) + amer_result_bytes(n); }

// American options by Longstaff-Schwartz: spill every option forward (which also clears its
// zero words), precompute the Gram factors of every date, run the backward inductions (as many
// options per cooperative launch as fit co-resident, each on its own blocks), finish all
// options with one launch and enqueue one read-back into the pinned staging at stage (the
// context's pinned buffer, at an offset that leaves amer_pinned_bytes(n) inside it).  Nothing is
// synchronised; *coop tells collect_american_group how the induction ran.
simr_status enqueue_american_group(simr_ctx* c, int scheme, const simr_option* opts, const AmerGroup& g,
                                   bool want_beta, char* stage, hipStream_t s, bool* coop_out) {
  const int n = (int)g.idx.size();
  if (stage < (char*)c->pinned || stage + amer_pinned_bytes(n) > (char*)c->pinned + c->pinned_bytes)
    return fail(SIMR_EINVAL, "internal: pinned staging too small");
  std::vector<DevOpt> d(n);
  std::vector<int64_t> paths(n);
  for (int k = 0; k < n; ++k) {
    simr_status st = devopt_for(c, scheme, opts[g.idx[k]], &d[k]);
    if (st != SIMR_OK) return st;
    paths[k] = opts[g.idx[k]].paths;
  }
  // first on the stream: the long forward passes hide the host's later enqueues (every launch
  // is its own profile record)
  for (int k = 0; k < n; ++k) {
    const int64_t nz = kOptZeroWords + (k == n - 1 ? 16 : 0);  // the last one also clears the status
    Prof pf(c, SIMR_PROF_SPILL, s);
    SIMR_HIP(launch_forward_spill(scheme, d[k], g.b[k].xs, g.b[k].vs, g.zero + (size_t)k * kOptZeroWords, nz, s));
  }
  std::vector<int> grids;
  std::vector<LsmLaunchSet> sets;
  if (!c->lsm_per_date) sets = lsm_coop_plan(paths, c->num_cus, c->lsm_grid_max, &grids, 6, c->lsm_block);
  const bool coop = !sets.empty();
  // the task table: the cooperative launches' blocks, and the finish's partial rows
  LsmTask* ht = (LsmTask*)stage;
  std::vector<int> block0(n, 0);
  for (const LsmLaunchSet& ls : sets) {
    int b0 = 0;
    for (int k = ls.first; k < ls.first + ls.count; ++k) {
      block0[k] = b0;
      b0 += grids[k];
    }
  }
  for (int k = 0; k < n; ++k) {
    const LsmBufs& b = g.b[k];
    LsmTask t;
    t.o = d[k];
    t.xs = b.xs;
    t.vs = b.vs;
    t.fac = b.fac;
    t.tau = b.tau;
    t.xchg = b.xchg;
    t.partials = b.partials;
    t.beta64 = want_beta ? b.st.beta64 : nullptr;
    t.flags = b.st.flags;
    t.block0 = block0[k];
    t.nblocks = coop ? grids[k] : b.nblk;
    ht[k] = t;
  }
  SIMR_HIP(hipMemcpyAsync(g.tasks, ht, sizeof(LsmTask) * (size_t)n, hipMemcpyHostToDevice, s));
  if (coop) {
    if (c->lsm_fail_test) SIMR_HIP(hipMemsetD32Async((hipDeviceptr_t)g.status, 1u, 1, s));
    for (int k = 0; k < n; ++k) {
      Prof pf(c, SIMR_PROF_GRAM, s);
      SIMR_HIP(launch_lsm_gram(d[k], g.b[k].xs, g.b[k].vs, g.b[k].gram, s));
    }
    for (int k = 0; k < n; ++k) {
      Prof pf(c, SIMR_PROF_FACTOR, s);
      SIMR_HIP(launch_lsm_factor(d[k], opts[g.idx[k]].r * opts[g.idx[k]].T / opts[g.idx[k]].steps, g.b[k].gram,
                                 g.b[k].fac, g.b[k].st.flags, s));
    }
    for (const LsmLaunchSet& ls : sets) {
      Prof pf(c, SIMR_PROF_LSM, s);
      SIMR_HIP(launch_lsm_coop(g.tasks + ls.first, ls.count, ls.block, ls.ppl, ls.grid, g.status, s));
    }
  } else {
    Prof pf(c, SIMR_PROF_LSM, s);
    for (int k = 0; k < n; ++k)
      SIMR_HIP(launch_lsm(d[k], g.b[k].xs, g.b[k].vs, g.b[k].hcash, g.b[k].tau, g.b[k].st, g.b[k].partials, s));
  }
  SIMR_HIP(launch_finalize_tasks(g.tasks, n, g.status, g.results, s));
  SIMR_HIP(hipMemcpyAsync(stage + amer_task_bytes(n), g.results, amer_result_bytes(n), hipMemcpyDeviceToHost, s));
  *coop_out = coop;
  return SIMR_OK;
}

// After the stream has been synchronised: the results of an enqueued pass.  out[k] receives the
// result of option g.idx[k].
simr_status collect_american_group(const simr_option* opts, const AmerGroup& g, bool coop, const char* stage,
                                   simr_result* out) {
  const int n = (int)g.idx.size();
  const double* sums = (const double*)(stage + amer_task_bytes(n));
  const int32_t* fl = (const int32_t*)(sums + 2 * n);
  if (coop && fl[n] != 0) return fail(SIMR_ENUMERIC, "Longstaff-Schwartz exchange wait timed out");
  for (int k = 0; k < n; ++k) {
    const simr_option& o = opts[g.idx[k]];
    double mean, se;
    mean_se(sums[2 * k], sums[2 * k + 1], o.paths, &mean, &se);
    simr_result r;
    std::memset(&r, 0, sizeof r);
    int32_t flags = fl[k];
    const double h0 = intrinsic_host(o, o.S0);
    // mean already discounts each cash flow to t_0: e^{-r tau dt} h
    if (h0 > mean) {
      r.price = h0;
      r.std_err = 0.0;
      flags |= SIMR_LSM_EXERCISE_T0;
    } else {
      r.price = mean;
      r.std_err = se;
    }
    r.paths = o.paths;
    r.lsm_flags = flags;
    out[k] = r;
  }
  return SIMR_OK;
}

simr_status run_american_group(simr_ctx* c, int scheme, const simr_option* opts, const AmerGroup& g,
                               simr_result* out, bool want_beta, hipStream_t s) {
  simr_status st = ensure_pinned(c, amer_pinned_bytes((int)g.idx.size()));
  if (st != SIMR_OK) return st;
  bool coop = false;
  if ((st = enqueue_american_group(c, scheme, opts, g, want_beta, (char*)c->pinned, s, &coop)) != SIMR_OK) return st;
  SIMR_HIP(hipStreamSynchronize(s));
  return collect_american_group(opts, g, coop, (const char*)c->pinned, out);
}


// Workspace of a group of American options in a Greeks batch (defined with the batch).
size_t greeks_group_bytes(const simr_option* opts, int64_t first, int64_t count, int ck);
}  // namespace

// =============================================================================================
// C ABI
// =============================================================================================
extern "C" {

const char* simr_status_string(simr_status s) {
  switch (s) {
    case SIMR_OK: return "ok";
    case SIMR_EINVAL: return "invalid argument";
    case SIMR_ENOMEM: return "out of host memory";
    case SIMR_EHIP: return "HIP runtime error";
    case SIMR_EUNSUPPORTED: return "unsupported";
    case SIMR_ENUMERIC: return "numerical failure";
  }
  return "unknown status";
}

const char* simr_last_error(void) { return g_err.c_str(); }

simr_status simr_create(simr_ctx** ctx, int device) {
  if (!ctx) return fail(SIMR_EINVAL, "ctx is NULL");
  FaultPlan plan;
  if (const char* e = std::getenv("SIMR_FAULT_INJECT")) {
    if (!parse_fault(e, &plan))
      return fail(SIMR_EINVAL, "SIMR_FAULT_INJECT=\"%s\": expected alloc, launch, sync or create, optionally "
                               "followed by :n with n >= 1", e);
    if (plan.kind == kFaultCreate) return fail(SIMR_EHIP, "injected create failure: no HIP call made");
  }
  int ndev = 0;
  SIMR_HIP(hipGetDeviceCount(&ndev));
  if (device < 0 || device >= ndev) return fail(SIMR_EINVAL, "device %d out of range (%d devices)", device, ndev);
  hipDeviceProp_t prop;
  SIMR_HIP(hipGetDeviceProperties(&prop, device));
  simr_ctx* c = new (std::nothrow) simr_ctx();
  if (!c) return fail(SIMR_ENOMEM, "context allocation failed");
  c->device = device;
  c->fault = plan;
  c->num_cus = prop.multiProcessorCount;
  if (const char* e = std::getenv("SIMR_LSM_GRID_MAX")) c->lsm_grid_max = std::max(1, std::atoi(e));
  if (const char* e = std::getenv("SIMR_LSM_PER_DATE")) c->lsm_per_date = std::atoi(e) != 0;
  c->arch = prop.gcnArchName;
  const std::string a = c->arch.substr(0, c->arch.find(':'));
  if (a != "gfx950") {
    delete c;
    return fail(SIMR_EUNSUPPORTED, "device %d is %s; this library is built for gfx950", device, prop.gcnArchName);
  }
  // The context's only device allocation: the truncated Gaussian table (128 KiB), built here so
  // that no pricing or Greeks call allocates device memory.  Then the device address of this
  // device's static scratch array (the allocation-free entry point's buffer), and the pinned
  // host words its result sums are copied to.
  simr_status st;
  {
    DeviceGuard g(device);
    st = build_tg_table(c);
    if (st == SIMR_OK) {
      void* ptr = nullptr;
      const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
      if (e != hipSuccess || !ptr)
        st = fail(SIMR_EHIP, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
      c->scratch = (char*)ptr;
    }
    if (st == SIMR_OK) {
      void* h = nullptr;
      const hipError_t e = hipHostMalloc(&h, 64, hipHostMallocDefault);
      if (e != hipSuccess || !h) st = fail(SIMR_EHIP, "hipHostMalloc(64 B): %s", hipGetErrorString(e));
      c->noalloc_sums = (double*)h;
    }
  }
  if (st != SIMR_OK) {
    DeviceGuard g(device);
    if (c->tg) (void)hipFree(c->tg);
    if (c->noalloc_sums) (void)hipHostFree(c->noalloc_sums);
    delete c;
    return st;
  }
  *ctx = c;
  return SIMR_OK;
}

simr_status simr_destroy(simr_ctx* ctx) {
  if (!ctx) return SIMR_OK;
  DeviceGuard g(ctx);
  for (auto& kv : ctx->graphs) (void)hipGraphExecDestroy(kv.second.exec);
  for (auto& pr : ctx->prof_pending) {
    (void)hipEventDestroy(pr.a);
    (void)hipEventDestroy(pr.b);
  }
  for (hipEvent_t e : ctx->prof_pool) (void)hipEventDestroy(e);
  if (ctx->pinned) (void)hipHostFree(ctx->pinned);
  if (ctx->noalloc_sums) (void)hipHostFree(ctx->noalloc_sums);
  if (ctx->tg) (void)hipFree(ctx->tg);
  delete ctx;
  return SIMR_OK;
}

simr_status simr_profile_enable(simr_ctx* ctx, int on) {
  if (!ctx) return fail(SIMR_EINVAL, "ctx is NULL");
  ctx->prof_on = on != 0;
  return SIMR_OK;
}

simr_status simr_profile_groups(simr_ctx* ctx, uint32_t mask) {
  if (!ctx) return fail(SIMR_EINVAL, "ctx is NULL");
  if (mask == 0 || (mask >> SIMR_PROF_GROUPS) != 0)
    return fail(SIMR_EINVAL, "group mask 0x%x: expected a nonzero mask of the %d groups", mask, SIMR_PROF_GROUPS);
  ctx->prof_mask = mask;
  return SIMR_OK;
}

simr_status simr_profile_read(simr_ctx* ctx, int group, double* total_ms, int64_t* launches) {
  if (!ctx || !total_ms || !launches) return fail(SIMR_EINVAL, "NULL argument");
  if (group < 0 || group >= SIMR_PROF_GROUPS) return fail(SIMR_EINVAL, "unknown profile group %d", group);
  DeviceGuard g(ctx);
  for (auto& pr : ctx->prof_pending) {
    SIMR_HIP(hipEventSynchronize(pr.b));
    float ms = 0;
    SIMR_HIP(hipEventElapsedTime(&ms, pr.a, pr.b));
    ctx->prof_ms[pr.group] += ms;
    ctx->prof_n[pr.group] += 1;
    ctx->prof_pool.push_back(pr.a);
    ctx->prof_pool.push_back(pr.b);
  }
  ctx->prof_pending.clear();
  *total_ms = ctx->prof_ms[group];
  *launches = ctx->prof_n[group];
  return SIMR_OK;
}

simr_status simr_profile_reset(simr_ctx* ctx) {
  if (!ctx) return fail(SIMR_EINVAL, "ctx is NULL");
  double ms;
  int64_t n;
  simr_status st = simr_profile_read(ctx, 0, &ms, &n);  // drains pending events
  if (st != SIMR_OK) return st;
  for (int i = 0; i < SIMR_PROF_GROUPS; ++i) {
    ctx->prof_ms[i] = 0;
    ctx->prof_n[i] = 0;
  }
  return SIMR_OK;
}

simr_status simr_set_lsm_launch(simr_ctx* ctx, int32_t mode, int32_t grid_max) {
  if (!ctx) return fail(SIMR_EINVAL, "ctx is NULL");
  if (mode < 0 || mode > 4)
    return fail(SIMR_EINVAL, "mode must be 0 (cooperative), 1 (one launch per date), 2 (failure test), 3 "
                             "(cooperative on 256-thread blocks) or 4 (cooperative on 1024-thread blocks)");
  if (grid_max < 0) return fail(SIMR_EINVAL, "grid_max must be >= 0");
  ctx->lsm_per_date = mode == 1;
  ctx->lsm_fail_test = mode == 2;
  ctx->lsm_block = mode == 3 ? 256 : mode == 4 ? 1024 : 0;
  if (grid_max > 0) ctx->lsm_grid_max = grid_max;
  return SIMR_OK;
}

simr_status simr_debug_fault(simr_ctx* ctx, int32_t kind, int32_t nth, int64_t* fired) {
  if (!ctx) return fail(SIMR_EINVAL, "ctx is NULL");
  if (kind < 0 || kind > kFaultSync) return fail(SIMR_EINVAL, "fault kind %d is not 0 (off), 1 (alloc), 2 (launch) "
                                                              "or 3 (sync)", kind);
  if (kind != 0 && nth < 1) return fail(SIMR_EINVAL, "nth must be >= 1");
  if (fired) *fired = ctx->fault.fired;
  ctx->fault.kind = kind;
  ctx->fault.countdown = kind ? nth : 0;
  return SIMR_OK;
}

simr_status simr_debug_graph_stats(simr_ctx* ctx, int64_t* captures, int64_t* launches) {
  if (!ctx || !captures || !launches) return fail(SIMR_EINVAL, "NULL argument");
  *captures = ctx->graph_captures;
  *launches = ctx->graph_launches;
  return SIMR_OK;
}

simr_status simr_get_tile(simr_ctx* ctx, int32_t* block, int32_t* ppl) {
  if (!ctx || !block || !ppl) return fail(SIMR_EINVAL, "NULL argument");
  *block = ctx->tile_block[0];
  *ppl = ctx->tile_ppl[0];
  return SIMR_OK;
}

simr_status simr_set_tile(simr_ctx* ctx, int32_t block, int32_t ppl) {
  if (!ctx) return fail(SIMR_EINVAL, "ctx is NULL");
  bool ok = false;
  for (auto& cand : kCandidates) ok |= (cand[0] == block && cand[1] == ppl);
  if (!ok) return fail(SIMR_EINVAL, "tile (%d, %d) is not a compiled candidate", block, ppl);
  for (int s = 0; s < (int)(sizeof(ctx->tile_block) / sizeof(ctx->tile_block[0])); ++s) {
    ctx->tile_block[s] = block;
    ctx->tile_ppl[s] = ppl;
  }
  return SIMR_OK;
}

simr_status simr_workspace_size(simr_ctx* ctx, int op, const simr_option* opts, int64_t n, const simr_params* params,
                                size_t* bytes) {
  (void)ctx;  // the sizes depend on the arguments only
  if (!bytes) return fail(SIMR_EINVAL, "bytes is NULL");
  int scheme, ck;
  simr_status st = validate_params(params, &scheme, &ck);
  if (st != SIMR_OK) return st;
  if (!opts || n < 1) return fail(SIMR_EINVAL, "need at least one option");
  if ((op == 0 || op == 2) && n != 1) return fail(SIMR_EINVAL, "ops 0 and 2 take one option");
  for (int64_t i = 0; i < n; ++i)
    if ((st = validate_option(&opts[i], i)) != SIMR_OK) return st;
  if (op == 0 || op == 1) {
    *bytes = batch_bytes(opts, n, kMinTilePaths);  // the smallest tile gives the most units
    return SIMR_OK;
  }
  if (op == 2) {
    Carve one(nullptr);
    if (american(opts[0])) carve_amer_group(one, opts, {0});
    carve_greeks_euro(one, opts[0].paths, opts[0].steps, ck);
    *bytes = one.off;
    return SIMR_OK;
  }
  if (op == 3) {
    // the options one after another in one workspace, American ones in groups of consecutive
    // options of at most kAmerPassBytes together (or one alone); a smaller workspace, down to
    // the largest single option's, makes smaller groups
    size_t most = 0;
    for (int64_t i = 0; i < n;) {
      int64_t m = 1;
      if (american(opts[i])) {
        while (i + m < n && m < 1024 && american(opts[i + m]) &&
               greeks_group_bytes(opts, i, m + 1, ck) <= std::max(kAmerPassBytes, greeks_group_bytes(opts, i, 1, ck)))
          ++m;
        most = std::max(most, greeks_group_bytes(opts, i, m, ck));
      } else {
        Carve one(nullptr);
        carve_greeks_euro(one, opts[i].paths, opts[i].steps, ck);
        most = std::max(most, one.off);
      }
      i += m;
    }
    *bytes = most;
    return SIMR_OK;
  }
  return fail(SIMR_EINVAL, "unknown op %d", op);
}

simr_status simr_price_batch(simr_ctx* ctx, const simr_option* opts, int64_t n, const simr_params* params,
                             simr_result* out, void* d_ws, size_t ws_bytes, void* stream) {
  if (!opts || !out || n < 1) return fail(SIMR_EINVAL, "NULL argument or n < 1");
  int scheme, ck;
  simr_status st = validate_params(params, &scheme, &ck);
  if (st != SIMR_OK) return st;
  for (int64_t i = 0; i < n; ++i)
    if ((st = validate_option(&opts[i], i)) != SIMR_OK) return st;
  if (!ctx) return fail(SIMR_EINVAL, "ctx is NULL");
  const size_t need = batch_bytes(opts, n, kMinTilePaths);
  if (!d_ws || ws_bytes < need) return fail(SIMR_EINVAL, "workspace too small: %zu < %zu bytes", ws_bytes, need);
  DeviceGuard g(ctx);
  hipStream_t s = (hipStream_t)stream;
  std::vector<simr_result> res(n);
  Carve cv(d_ws);
  TuneBufs tb = carve_tune(cv);
  BatchPlan pl0 = plan_batch(opts, n, kMinTilePaths);
  if (!pl0.euro.empty() && (st = autotune(ctx, scheme, tb, s)) != SIMR_OK) return st;
  const int tile = (ctx->tile_block[scheme] ? ctx->tile_block[scheme] * ctx->tile_ppl[scheme] : kMinTilePaths);
  BatchPlan pl = plan_batch(opts, n, tile);
  BatchBufs bb = carve_batch(cv, (int64_t)pl.euro.size(), pl.total_tiles);
  if ((st = run_euro_batch(ctx, scheme, opts, pl.euro, bb, pl.total_tiles, res.data(), s)) != SIMR_OK) return st;
  for (const auto& grp : amer_passes(opts, pl.amer)) {
    Carve cg = cv;  // every pass reuses the same region
    AmerGroup ag = carve_amer_group(cg, opts, grp);
    std::vector<simr_result> r(grp.size());
    if ((st = run_american_group(ctx, scheme, opts, ag, r.data(), false, s)) != SIMR_OK) return st;
    for (size_t k = 0; k < grp.size(); ++k) res[grp[k]] = r[k];
  }
  std::memcpy(out, res.data(), sizeof(simr_result) * (size_t)n);
  return SIMR_OK;
}

simr_status simr_price(simr_ctx* ctx, const simr_option* opt, const simr_params* params, simr_result* out, void* d_ws,
                       size_t ws_bytes, void* stream) {
  if (!opt || !out) return fail(SIMR_EINVAL, "NULL argument");
  return simr_price_batch(ctx, opt, 1, params, out, d_ws, ws_bytes, stream);
}

simr_status simr_price_noalloc(simr_ctx* ctx, const simr_option* opt, const simr_params* params, simr_result* out,
                               void* stream) {
  if (!opt || !out) return fail(SIMR_EINVAL, "NULL argument");
  int scheme, ck;
  simr_status st = validate_params(params, &scheme, &ck);
  if (st != SIMR_OK) return st;
  if ((st = validate_option(opt, 0)) != SIMR_OK) return st;
  if (american(*opt))
    return fail(SIMR_EUNSUPPORTED, "simr_price_noalloc prices European options only (an American option needs "
                                   "its path states in a caller workspace: simr_price)");
  if (!ctx) return fail(SIMR_EINVAL, "ctx is NULL");
  if (!ctx->scratch || !ctx->noalloc_sums) return fail(SIMR_EINVAL, "internal: the context has no scratch address");
  int block = ctx->tile_block[scheme], ppl = ctx->tile_ppl[scheme];
  if (!block) {  // not tuned on this context: a fixed compiled tile, no timing runs
    block = 256;
    ppl = 1;
  }
  const int64_t tile = (int64_t)block * ppl;
  const int64_t ntiles = (opt->paths + tile - 1) / tile;
  if (ntiles > kScratchTiles)
    return fail(SIMR_EINVAL, "option needs %lld path tiles of %lld paths; the static scratch holds %lld tiles "
                             "(at most %lld paths at this tile)", (long long)ntiles, (long long)tile,
                (long long)kScratchTiles, (long long)(kScratchTiles * tile));
  DeviceGuard g(ctx);
  hipStream_t s = (hipStream_t)stream;
  // the record: the option's constants, then order {0} and the unit prefix {0, ntiles}
  alignas(8) unsigned char rec[kScratchRecord];
  std::memset(rec, 0, sizeof rec);
  DevOpt d;
  if ((st = devopt_for(ctx, scheme, *opt, &d)) != SIMR_OK) return st;
  d.slot0 = 0;
  d.ntiles = (int32_t)ntiles;
  std::memcpy(rec, &d, sizeof d);
  const int32_t tail[3] = {0, 0, (int32_t)ntiles};
  std::memcpy(rec + 512, tail, sizeof tail);
  char* base = ctx->scratch;
  BatchLaunch L;
  L.opts = (const DevOpt*)base;
  L.order = (const int32_t*)(base + 512);
  L.uprefix = (const int32_t*)(base + 516);
  L.nopt = 1;
  L.nunits = (int32_t)ntiles;
  L.counter = (uint32_t*)(base + kScratchCounter);
  L.partials = (double*)(base + kScratchPartials);
  L.block = block;
  L.ppl = ppl;
  L.grid = grid_for(ctx, scheme, block, ppl, ntiles);
  double* results = (double*)(base + kScratchResult);
  SIMR_HIP(launch_stage_record(rec, sizeof rec, base, s));
  SIMR_HIP(launch_reset_words(L.counter, 16, s));
  SIMR_HIP(launch_batch_price(scheme, L, s));
  SIMR_HIP(launch_finalize_rows(L.partials, 2, L.opts, 1, 0, results, s));
  double* h = ctx->noalloc_sums;  // pinned at simr_create: the copy needs no staging of its own
  SIMR_HIP(hipMemcpyAsync(h, results, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
  SIMR_HIP(hipStreamSynchronize(s));
  simr_result r;
  std::memset(&r, 0, sizeof r);
  mean_se(h[0], h[1], opt->paths, &r.price, &r.std_err);
  r.paths = opt->paths;
  *out = r;
  return SIMR_OK;
}

}  // extern "C"

namespace {

// The Greeks of one option: ng = 7 (simr_greeks) or 9 (simr_greeks_ext: also d/dT and gamma).
// greeks_check validates what needs no device, greeks_enqueue puts the whole computation on the
// stream with its read-back into the pinned staging at stage (greeks_stage_bytes), and
// greeks_collect turns the staged sums into the outputs once the stream has been synchronised.

// Pinned staging of one option: [American pass staging | 2 + 2 ng doubles of sums].
size_t greeks_sums_offset(bool am) { return am ? (amer_pinned_bytes(1) + 63) / 64 * 64 : 0; }
size_t greeks_stage_bytes(bool am) {
  return (greeks_sums_offset(am) + kGreekResultDoubles * sizeof(double) + 63) / 64 * 64;
}

simr_status greeks_check(const simr_option* opt, const simr_params* params, int64_t i, int* scheme, int* ck) {
  simr_status st = validate_params(params, scheme, ck);
  if (st != SIMR_OK) return st;
  if ((st = validate_option(opt, i)) != SIMR_OK) return st;
  if (*scheme == SIMR_SCHEME_BK)
    return fail(SIMR_EUNSUPPORTED, "adjoint Greeks are not implemented for the Broadie-Kaya scheme");
  return SIMR_OK;
}

struct GreeksPending {
  bool am = false;
  bool coop = false;
  AmerGroup ag;
};

simr_status greeks_enqueue(simr_ctx* ctx, const simr_option* opt, int scheme, int ck, int ng, void* d_ws, char* stage,
                           hipStream_t s, GreeksPending* pend) {
  const simr_option& o = *opt;
  const bool ext = ng > SIMR_NUM_GREEKS;
  DevOpt d;
  simr_status st = devopt_for(ctx, scheme, o, &d);  // the TG table attached
  if (st != SIMR_OK) return st;
  Carve cv(d_ws);
  pend->am = american(o);
  if (pend->am) pend->ag = carve_amer_group(cv, opt, {0});
  GreekBufs gb = carve_greeks_euro(cv, o.paths, o.steps, ck);
  const int ablock = adjoint_block(o.paths, ck, ext, ctx->num_cus);
  if (pend->am) {
    // the adjoint is enqueued right behind the induction (no host round trip); if the option
    // turns out to be exercised at t_0 its sums are simply not used
    if ((st = enqueue_american_group(ctx, scheme, opt, pend->ag, false, stage, s, &pend->coop)) != SIMR_OK) return st;
    const LsmBufs& lb = pend->ag.b[0];
    Prof pf(ctx, SIMR_PROF_ADJOINT, s);
    SIMR_HIP(launch_adjoint(scheme, d, ck, ablock, ext, lb.vs + (size_t)(ck - 1) * o.paths, (size_t)ck * o.paths,
                            lb.xs, lb.tau, gb.gpart, s));
  } else {
    {
      Prof pf(ctx, SIMR_PROF_CKPT, s);
      SIMR_HIP(launch_forward_ckpt(scheme, d, ck, gb.ck, gb.xN, gb.partials, s));
    }
    SIMR_HIP(launch_finalize_rows(gb.partials, 2, nullptr, 1, gb.nblk, gb.result, s));
    Prof pf(ctx, SIMR_PROF_ADJOINT, s);
    SIMR_HIP(launch_adjoint(scheme, d, ck, ablock, ext, gb.ck, (size_t)o.paths, gb.xN, nullptr, gb.gpart, s));
  }
  SIMR_HIP(launch_finalize_rows(gb.gpart, 2 * ng, nullptr, 1, (int)((o.paths + ablock - 1) / ablock), gb.result + 2,
                                s));
  double* h = (double*)(stage + greeks_sums_offset(pend->am));
  SIMR_HIP(hipMemcpyAsync(h, gb.result, (2 + 2 * (size_t)ng) * sizeof(double), hipMemcpyDeviceToHost, s));
  return SIMR_OK;
}

// The Greeks from their staged sums h (2 price sums, then ng Greek sums and ng sums of squares);
// an American option exercised at t_0 takes those of its value h(S0), linear in S0.
void greeks_from_sums(const simr_option& o, int ng, const double* h, int32_t lsm_flags, double* g, double* g_se) {
  if (lsm_flags & SIMR_LSM_EXERCISE_T0) {
    for (int i = 0; i < ng; ++i) g[i] = g_se[i] = 0.0;
    g[0] = (o.payoff == SIMR_AMER_CALL) ? 1.0 : -1.0;
    return;
  }
  for (int i = 0; i < ng; ++i) mean_se(h[2 + i], h[2 + ng + i], o.paths, &g[i], &g_se[i]);
}

simr_status greeks_collect(const simr_option* opt, int ng, const char* stage, const GreeksPending& pend, double* price,
                           double* std_err, double* g, double* g_se, int32_t* lsm_flags) {
  const simr_option& o = *opt;
  const double* h = (const double*)(stage + greeks_sums_offset(pend.am));
  *lsm_flags = 0;
  if (pend.am) {
    simr_result pr;
    simr_status st = collect_american_group(opt, pend.ag, pend.coop, stage, &pr);
    if (st != SIMR_OK) return st;
    *price = pr.price;
    *std_err = pr.std_err;
    *lsm_flags = pr.lsm_flags;
  } else {
    mean_se(h[0], h[1], o.paths, price, std_err);
  }
  greeks_from_sums(o, ng, h, *lsm_flags, g, g_se);
  return SIMR_OK;
}

// A Greeks batch as items: a European option alone, or a group of consecutive American options
// whose inductions share one cooperative launch and whose buffers fit the workspace together
// (their spills, Gram sums, factors and inductions enqueued as one pass, then the adjoint of
// each).  The launch shape of an option's induction does not change its bits, so neither does
// the grouping.
struct GreeksItem {
  int64_t first = 0, count = 1;
  bool am = false, coop = false;
  AmerGroup ag;
  size_t stage = 0;  // the item's staging in the pinned buffer: [American pass | sums of each option]
};

constexpr size_t kGreekSumsBytes = (kGreekResultDoubles * sizeof(double) + 63) / 64 * 64;

size_t greeks_item_sums_offset(const GreeksItem& it) {
  return it.am ? (amer_pinned_bytes((int)it.count) + 63) / 64 * 64 : 0;
}

// Workspace of an American group: the pass's buffers, then the adjoint's of its largest option
// (the options' adjoints run one after another).
size_t greeks_group_bytes(const simr_option* opts, int64_t first, int64_t count, int ck) {
  std::vector<int64_t> idx;
  int64_t P = 0;
  int N = 0;
  for (int64_t k = 0; k < count; ++k) {
    idx.push_back(first + k);
    P = std::max(P, opts[first + k].paths);
    N = std::max(N, opts[first + k].steps);
  }
  Carve cv(nullptr);
  carve_amer_group(cv, opts, idx);
  carve_greeks_euro(cv, P, N, ck);
  return cv.off;
}

std::vector<GreeksItem> greeks_plan(simr_ctx* ctx, const simr_option* opts, int64_t n, int ck, size_t ws_bytes) {
  std::vector<GreeksItem> items;
  size_t stage = 0;
  for (int64_t i = 0; i < n;) {
    GreeksItem it;
    it.first = i;
    it.am = american(opts[i]);
    if (it.am && !ctx->lsm_per_date) {
      // the options of the first cooperative launch of the run of American options from i (a
      // launch holds at most 1024 blocks, so at most 1024 options), as many as fit the workspace
      std::vector<int64_t> paths;
      for (int64_t k = i; k < n && k < i + 1024 && american(opts[k]); ++k) paths.push_back(opts[k].paths);
      std::vector<int> grids;
      const std::vector<LsmLaunchSet> sets = lsm_coop_plan(paths, ctx->num_cus, ctx->lsm_grid_max, &grids, 6,
                                                           ctx->lsm_block);
      it.count = sets.empty() ? 1 : sets[0].count;
      while (it.count > 1 && greeks_group_bytes(opts, i, it.count, ck) > ws_bytes) --it.count;
    }
    it.stage = stage;
    stage += greeks_item_sums_offset(it) + kGreekSumsBytes * (size_t)it.count;
    items.push_back(it);
    i += it.count;
  }
  return items;
}

simr_status greeks_enqueue_group(simr_ctx* ctx, const simr_option* opts, int scheme, int ck, int ng, void* d_ws,
                                 char* stage, hipStream_t s, GreeksItem* it) {
  const bool ext = ng > SIMR_NUM_GREEKS;
  std::vector<int64_t> idx;
  int64_t P = 0;
  int N = 0;
  for (int64_t k = 0; k < it->count; ++k) {
    idx.push_back(it->first + k);
    P = std::max(P, opts[it->first + k].paths);
    N = std::max(N, opts[it->first + k].steps);
  }
  Carve cv(d_ws);
  it->ag = carve_amer_group(cv, opts, idx);
  GreekBufs gb = carve_greeks_euro(cv, P, N, ck);
  simr_status st = enqueue_american_group(ctx, scheme, opts, it->ag, false, stage, s, &it->coop);
  if (st != SIMR_OK) return st;
  for (int64_t k = 0; k < it->count; ++k) {
    const simr_option& o = opts[it->first + k];
    DevOpt d;
    if ((st = devopt_for(ctx, scheme, o, &d)) != SIMR_OK) return st;
    const LsmBufs& lb = it->ag.b[(size_t)k];
    const int ablock = adjoint_block(o.paths, ck, ext, ctx->num_cus);
    {
      Prof pf(ctx, SIMR_PROF_ADJOINT, s);
      SIMR_HIP(launch_adjoint(scheme, d, ck, ablock, ext, lb.vs + (size_t)(ck - 1) * o.paths, (size_t)ck * o.paths,
                              lb.xs, lb.tau, gb.gpart, s));
    }
    SIMR_HIP(launch_finalize_rows(gb.gpart, 2 * ng, nullptr, 1, (int)((o.paths + ablock - 1) / ablock),
                                  gb.result + 2, s));
    double* h = (double*)(stage + greeks_item_sums_offset(*it) + kGreekSumsBytes * (size_t)k);
    SIMR_HIP(hipMemcpyAsync(h, gb.result, (2 + 2 * (size_t)ng) * sizeof(double), hipMemcpyDeviceToHost, s));
  }
  return SIMR_OK;
}

simr_status greeks_impl(simr_ctx* ctx, const simr_option* opt, const simr_params* params, int ng, double* price,
                        double* std_err, double* g, double* g_se, int32_t* lsm_flags, void* d_ws, size_t ws_bytes,
                        void* stream) {
  int scheme, ck;
  simr_status st = greeks_check(opt, params, 0, &scheme, &ck);
  if (st != SIMR_OK) return st;
  if (!ctx) return fail(SIMR_EINVAL, "ctx is NULL");
  size_t need = 0;
  if ((st = simr_workspace_size(ctx, 2, opt, 1, params, &need)) != SIMR_OK) return st;
  if (!d_ws || ws_bytes < need) return fail(SIMR_EINVAL, "workspace too small: %zu < %zu bytes", ws_bytes, need);
  DeviceGuard guard(ctx);
  hipStream_t s = (hipStream_t)stream;
  if ((st = ensure_pinned(ctx, greeks_stage_bytes(american(*opt)))) != SIMR_OK) return st;
  GreeksPending pend;
  if ((st = greeks_enqueue(ctx, opt, scheme, ck, ng, d_ws, (char*)ctx->pinned, s, &pend)) != SIMR_OK) return st;
  SIMR_HIP(hipStreamSynchronize(s));
  return greeks_collect(opt, ng, (const char*)ctx->pinned, pend, price, std_err, g, g_se, lsm_flags);
}

}  // namespace

extern "C" {

simr_status simr_greeks(simr_ctx* ctx, const simr_option* opt, const simr_params* params, simr_greeks_result* out,
                        void* d_ws, size_t ws_bytes, void* stream) {
  if (!opt || !out) return fail(SIMR_EINVAL, "NULL argument");
  simr_greeks_result r;
  std::memset(&r, 0, sizeof r);
  simr_status st = greeks_impl(ctx, opt, params, SIMR_NUM_GREEKS, &r.price, &r.std_err, r.g, r.g_se, &r.lsm_flags,
                               d_ws, ws_bytes, stream);
  if (st == SIMR_OK) *out = r;
  return st;
}

simr_status simr_greeks_ext(simr_ctx* ctx, const simr_option* opt, const simr_params* params,
                            simr_greeks_ext_result* out, void* d_ws, size_t ws_bytes, void* stream) {
  if (!opt || !out) return fail(SIMR_EINVAL, "NULL argument");
  simr_greeks_ext_result r;
  std::memset(&r, 0, sizeof r);
  simr_status st = greeks_impl(ctx, opt, params, SIMR_NUM_GREEKS_EXT, &r.price, &r.std_err, r.g, r.g_se,
                               &r.lsm_flags, d_ws, ws_bytes, stream);
  if (st == SIMR_OK) *out = r;
  return st;
}

simr_status simr_greeks_batch(simr_ctx* ctx, const simr_option* opts, int64_t n, const simr_params* params,
                              simr_greeks_result* out, void* d_ws, size_t ws_bytes, void* stream) {
  if (!opts || !out || n < 1) return fail(SIMR_EINVAL, "NULL argument or n < 1");
  int scheme = 0, ck = 0;
  simr_status st = SIMR_OK;
  for (int64_t i = 0; i < n; ++i)
    if ((st = greeks_check(&opts[i], params, i, &scheme, &ck)) != SIMR_OK) return st;
  if (!ctx) return fail(SIMR_EINVAL, "ctx is NULL");
  size_t need = 0;  // the largest single option's (smaller groups in a smaller workspace)
  for (int64_t i = 0; i < n; ++i) {
    size_t one = 0;
    if ((st = simr_workspace_size(ctx, 2, &opts[i], 1, params, &one)) != SIMR_OK) return st;
    need = std::max(need, one);
  }
  if (!d_ws || ws_bytes < need) return fail(SIMR_EINVAL, "workspace too small: %zu < %zu bytes", ws_bytes, need);
  DeviceGuard guard(ctx);
  hipStream_t s = (hipStream_t)stream;
  std::vector<GreeksItem> items = greeks_plan(ctx, opts, n, ck, ws_bytes);
  size_t total = 0;
  for (const GreeksItem& it : items)
    total = std::max(total, it.stage + greeks_item_sums_offset(it) + kGreekSumsBytes * (size_t)it.count);
  if ((st = ensure_pinned(ctx, total)) != SIMR_OK) return st;
  // every item on the stream behind the one before (they share the workspace, which stream
  // order makes safe), each reading back into its own staging; one synchronisation
  std::vector<GreeksPending> pend(items.size());
  for (size_t q = 0; q < items.size(); ++q) {
    GreeksItem& it = items[q];
    char* stage = (char*)ctx->pinned + it.stage;
    if (it.am && it.count > 1)
      st = greeks_enqueue_group(ctx, opts, scheme, ck, SIMR_NUM_GREEKS, d_ws, stage, s, &it);
    else
      st = greeks_enqueue(ctx, &opts[it.first], scheme, ck, SIMR_NUM_GREEKS, d_ws, stage, s, &pend[q]);
    if (st != SIMR_OK) {
      // the read-backs already enqueued still target the staging: let them land first
      (void)hipStreamSynchronize(s);
      return st;
    }
  }
  SIMR_HIP(hipStreamSynchronize(s));
  std::vector<simr_greeks_result> r((size_t)n);
  for (size_t q = 0; q < items.size(); ++q) {
    const GreeksItem& it = items[q];
    const char* stage = (const char*)ctx->pinned + it.stage;
    if (it.am && it.count > 1) {
      std::vector<simr_result> pr((size_t)it.count);
      if ((st = collect_american_group(opts, it.ag, it.coop, stage, pr.data())) != SIMR_OK) return st;
      for (int64_t k = 0; k < it.count; ++k) {
        simr_greeks_result& ri = r[(size_t)(it.first + k)];
        std::memset(&ri, 0, sizeof ri);
        ri.price = pr[(size_t)k].price;
        ri.std_err = pr[(size_t)k].std_err;
        ri.lsm_flags = pr[(size_t)k].lsm_flags;
        const double* h = (const double*)(stage + greeks_item_sums_offset(it) + kGreekSumsBytes * (size_t)k);
        greeks_from_sums(opts[it.first + k], SIMR_NUM_GREEKS, h, ri.lsm_flags, ri.g, ri.g_se);
      }
    } else {
      simr_greeks_result& ri = r[(size_t)it.first];
      std::memset(&ri, 0, sizeof ri);
      if ((st = greeks_collect(&opts[it.first], SIMR_NUM_GREEKS, stage, pend[q], &ri.price, &ri.std_err, ri.g,
                               ri.g_se, &ri.lsm_flags)) != SIMR_OK)
        return st;
    }
  }
  for (int64_t i = 0; i < n; ++i) out[i] = r[(size_t)i];
  return SIMR_OK;
}

simr_status simr_debug_draws(simr_ctx* ctx, uint64_t seed, uint32_t stream_id, int64_t path0, int64_t npaths,
                             int32_t step0, int32_t nsteps, uint32_t* d_words, float* d_unif, float* d_norm,
                             void* stream) {
  if (npaths < 1 || nsteps < 1 || path0 < 0 || step0 < 0 || path0 + npaths > ((int64_t)1 << 32) ||
      (int64_t)step0 + nsteps > ((int64_t)1 << 32) || npaths * nsteps > ((int64_t)1 << 31))
    return fail(SIMR_EINVAL, "bad draw window");
  if (!ctx) return fail(SIMR_EINVAL, "ctx is NULL");
  DeviceGuard g(ctx);
  SIMR_HIP(launch_debug_draws(seed, stream_id, path0, npaths, step0, nsteps, d_words, d_unif, d_norm,
                              (hipStream_t)stream));
  return SIMR_OK;
}

simr_status simr_debug_paths(simr_ctx* ctx, const simr_option* opt, const simr_params* params, float* d_xT,
                             float* d_vT, float* d_payoff, void* stream) {
  if (!opt) return fail(SIMR_EINVAL, "NULL argument");
  int scheme, ck;
  simr_status st = validate_params(params, &scheme, &ck);
  if (st != SIMR_OK) return st;
  if ((st = validate_option(opt, 0)) != SIMR_OK) return st;
  if (!ctx) return fail(SIMR_EINVAL, "ctx is NULL");
  DeviceGuard g(ctx);
  DevOpt d;
  if ((st = devopt_for(ctx, scheme, *opt, &d)) != SIMR_OK) return st;
  SIMR_HIP(launch_debug_paths(scheme, d, d_xT, d_vT, d_payoff, (hipStream_t)stream));
  return SIMR_OK;
}

simr_status simr_debug_lsm(simr_ctx* ctx, const simr_option* opt, const simr_params* params, simr_result* out,
                           int32_t* d_tau, double* d_beta, void* d_ws, size_t ws_bytes, void* stream) {
  if (!opt || !out) return fail(SIMR_EINVAL, "NULL argument");
  int scheme, ck;
  simr_status st = validate_params(params, &scheme, &ck);
  if (st != SIMR_OK) return st;
  if ((st = validate_option(opt, 0)) != SIMR_OK) return st;
  if (!american(*opt)) return fail(SIMR_EINVAL, "simr_debug_lsm needs an American option");
  if (!ctx) return fail(SIMR_EINVAL, "ctx is NULL");
  const size_t need = amer_group_bytes(opt, {0});
  if (!d_ws || ws_bytes < need) return fail(SIMR_EINVAL, "workspace too small: %zu < %zu bytes", ws_bytes, need);
  DeviceGuard g(ctx);
  hipStream_t s = (hipStream_t)stream;
  Carve cv(d_ws);
  AmerGroup ag = carve_amer_group(cv, opt, {0});
  const LsmBufs& lb = ag.b[0];
  // dates with no regression keep zero coefficients
  SIMR_HIP(hipMemsetAsync(lb.st.beta64, 0, sizeof(double) * 6 * (size_t)(opt->steps + 1), s));
  if ((st = run_american_group(ctx, scheme, opt, ag, out, true, s)) != SIMR_OK) return st;
  if (d_tau) SIMR_HIP(hipMemcpyAsync(d_tau, lb.tau, sizeof(int32_t) * (size_t)opt->paths, hipMemcpyDeviceToDevice, s));
  if (d_beta)
    SIMR_HIP(hipMemcpyAsync(d_beta, lb.st.beta64, sizeof(double) * 6 * (size_t)(opt->steps + 1),
                            hipMemcpyDeviceToDevice, s));
  SIMR_HIP(hipStreamSynchronize(s));
  return SIMR_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------------------------
// Correlated baskets.
// ---------------------------------------------------------------------------------------------
namespace {

// Workspace sizes are computed without a context: sized for the larger block count of either
// launch layout (the split layout has up to 32x the blocks), whatever the device.
constexpr int kWorkspaceCus = 1 << 20;

bool basket_american(const simr_basket& b) { return b.payoff == SIMR_AMER_PUT || b.payoff == SIMR_AMER_CALL; }

// Asset i of the basket as a single option: its own Heston parameters, the basket's terms.
simr_option basket_asset(const simr_basket& b, int i) {
  simr_option o;
  std::memset(&o, 0, sizeof o);
  o.S0 = b.S0[i];
  o.K = b.K;
  o.T = b.T;
  o.r = b.r;
  o.kappa = b.kappa[i];
  o.theta = b.theta[i];
  o.xi = b.xi[i];
  o.rho = b.rho[i];
  o.v0 = b.v0[i];
  o.payoff = b.payoff;
  o.steps = b.steps;
  o.paths = b.paths;
  o.seed = b.seed;
  o.stream_id = b.stream_id;
  return o;
}

double basket_b0(const simr_basket& b) {
  double s = 0.0;
  for (int i = 0; i < b.assets; ++i) s += b.w[i] * b.S0[i];
  return s;
}

double corr_at(const simr_basket& b, int i, int j) { return b.corr[i * SIMR_MAX_ASSETS + j]; }

// Lower Cholesky factor of C in FP64 (L[i * d + j]); false if a pivot is <= 1e-12.
bool corr_factor(const simr_basket& b, std::vector<double>* L) {
  const int d = b.assets;
  L->assign((size_t)d * d, 0.0);
  for (int i = 0; i < d; ++i)
    for (int j = 0; j <= i; ++j) {
      double s = corr_at(b, i, j);
      for (int k = 0; k < j; ++k) s -= (*L)[i * d + k] * (*L)[j * d + k];
      if (i == j) {
        if (!(s > 1e-12)) return false;
        (*L)[i * d + i] = std::sqrt(s);
      } else {
        (*L)[i * d + j] = s / (*L)[j * d + j];
      }
    }
  return true;
}

simr_status validate_basket(const simr_basket* b) {
  if (!b) return fail(SIMR_EINVAL, "basket is NULL");
  if (b->assets < 1 || b->assets > SIMR_MAX_ASSETS)
    return fail(SIMR_EINVAL, "basket assets must be in [1, %d]", SIMR_MAX_ASSETS);
  if (b->reserved0 != 0 || b->reserved1 != 0) return fail(SIMR_EINVAL, "basket reserved fields must be 0");
  const int d = b->assets;
  for (int i = 0; i < d; ++i) {
    const simr_option o = basket_asset(*b, i);
    simr_status st = validate_option(&o, i);
    if (st != SIMR_OK) return st;
    if (!finite(b->w[i]) || b->w[i] < 0.0) return fail(SIMR_EINVAL, "basket weight %d must be finite and >= 0", i);
  }
  if (!(basket_b0(*b) > 0.0)) return fail(SIMR_EINVAL, "basket value sum w_i S0_i must be > 0");
  for (int i = 0; i < d; ++i)
    for (int j = 0; j < d; ++j) {
      const double c = corr_at(*b, i, j);
      if (!finite(c) || std::fabs(c) > 1.0) return fail(SIMR_EINVAL, "corr[%d][%d] must be finite in [-1, 1]", i, j);
      if (std::fabs(c - corr_at(*b, j, i)) > 1e-12) return fail(SIMR_EINVAL, "corr must be symmetric");
      if (i == j && std::fabs(c - 1.0) > 1e-12) return fail(SIMR_EINVAL, "corr must have a unit diagonal");
    }
  std::vector<double> L;
  if (!corr_factor(*b, &L)) return fail(SIMR_EINVAL, "corr is not positive definite");
  return SIMR_OK;
}

DevBasket make_devbasket(const simr_basket& b) {
  DevBasket k;
  std::memset(&k, 0, sizeof k);
  const int d = b.assets;
  k.d = d;
  k.steps = b.steps;
  k.paths = (int32_t)b.paths;
  k.payoff = b.payoff;
  k.stream = b.stream_id;
  k.seed_lo = (uint32_t)(b.seed & 0xffffffffu);
  k.seed_hi = (uint32_t)(b.seed >> 32);
  k.K = (float)b.K;
  k.disc = (float)std::exp(-b.r * b.T);
  k.rdt = (float)(b.r * b.T / b.steps);
  k.invB0 = (float)(1.0 / basket_b0(b));
  for (int i = 0; i < d; ++i) {
    k.w[i] = (float)b.w[i];
    k.wS0[i] = (float)(b.w[i] * b.S0[i]);
    k.S0[i] = (float)b.S0[i];
  }
  std::vector<double> L;
  corr_factor(b, &L);  // validated
  // W = L^{-1}, column by column: L W[:, c] = e_c
  std::vector<double> W((size_t)d * d, 0.0);
  for (int c = 0; c < d; ++c) {
    W[c * d + c] = 1.0 / L[c * d + c];
    for (int r = c + 1; r < d; ++r) {
      double t = 0.0;
      for (int q = c; q < r; ++q) t += L[r * d + q] * W[q * d + c];
      W[r * d + c] = -t / L[r * d + r];
    }
  }
  for (int i = 0; i < d; ++i)
    for (int j = 0; j <= i; ++j) {
      k.L[i * (i + 1) / 2 + j] = (float)L[i * d + j];
      k.Linv[i * (i + 1) / 2 + j] = (float)W[i * d + j];
    }
  return k;
}

int basket_ncol(int d) { return 2 + 2 * d + d * (d + 1); }
// Risk records per path: the cash flow, d vegas in v0, d in theta, d (d - 1) / 2 correlations.
int risk_cols(int d) { return 1 + 2 * d + d * (d - 1) / 2; }

// The derivative of the lower Cholesky factor L of C (L L^T = C) when C_ij and C_ji move
// together (i != j): from d(L L^T) = dL L^T + L dL^T, L^{-1} dC L^{-T} = X + X^T with X = L^{-1} dL
// lower triangular, so dL = L Phi(L^{-1} dC L^{-T}), Phi keeping the lower triangle and half the
// diagonal.  L^{-1} dC L^{-T} = a b^T + b a^T with a, b the columns i and j of L^{-1}.  FP64.
void chol_derivative(int d, const std::vector<double>& L, int i, int j, double* dL) {
  std::vector<double> W((size_t)d * d, 0.0);  // L^{-1} by forward substitution, column by column
  for (int c = 0; c < d; ++c)
    for (int r = c; r < d; ++r) {
      double t = r == c ? 1.0 : 0.0;
      for (int k = c; k < r; ++k) t -= L[r * d + k] * W[k * d + c];
      W[r * d + c] = t / L[r * d + r];
    }
  std::vector<double> Phi((size_t)d * d, 0.0);
  for (int r = 0; r < d; ++r)
    for (int c = 0; c <= r; ++c) {
      const double m = W[r * d + i] * W[c * d + j] + W[r * d + j] * W[c * d + i];
      Phi[r * d + c] = r == c ? 0.5 * m : m;
    }
  for (int r = 0; r < d; ++r)
    for (int c = 0; c <= r; ++c) {
      double t = 0.0;
      for (int k = c; k <= r; ++k) t += L[r * d + k] * Phi[k * d + c];
      dL[r * d + c] = t;
    }
}

// Workspace of one basket call: [DevBasket | DevOpt per asset | LsmTask] (uploaded from the
// pinned staging), the European block sums, the Greeks records and chunk moments, and for
// American baskets the write-out and the Longstaff-Schwartz buffers of the 10-function basis.
struct BasketBufs {
  char* upload;
  size_t upload_bytes, off_opts, off_task, off_dl;  // off_dl: the risk Greeks' Cholesky derivatives
  DevBasket* bk;
  DevOpt* ao;
  LsmTask* task;
  double* rows;      // 2 per block of 256 paths
  double* sums;      // column sums (2, or the Greeks' ncol)
  float* rec;        // Greeks records, (1 + 2 d) columns of P floats (risk: risk_cols(d))
  float* dl;         // risk Greeks: d L / d C_ij of every pair, kRiskTri floats each (in the upload)
  double* part;      // Greeks chunk moments
  float *xs, *vs, *gram;
  int32_t* tau;
  double *fac, *partials, *beta64, *results;
  float *wcash, *gpart, *beta32;  // the per-date induction (paths beyond the cooperative capacity)
  uint32_t* zero;    // [0] unused, [1] flags, [2] status, [3] per-date ticket, [16 ...) exchange words
  int64_t zero_words;
  int nblk, nchunk;
  int lpp;           // lanes per path of the basket kernels
};

BasketBufs carve_basket(Carve& cv, const simr_basket& b, int op, int num_cus) {
  BasketBufs u;
  std::memset(&u, 0, sizeof u);
  const int d = b.assets;
  const int64_t P = b.paths;
  const int N = b.steps;
  u.off_opts = (sizeof(DevBasket) + kAlign - 1) / kAlign * kAlign;
  u.off_task = u.off_opts + (sizeof(DevOpt) * (size_t)d + kAlign - 1) / kAlign * kAlign;
  u.off_dl = (u.off_task + sizeof(LsmTask) + kAlign - 1) / kAlign * kAlign;
  u.upload_bytes = op == 3 ? u.off_dl + sizeof(float) * (size_t)kRiskPairs * kRiskTri : u.off_task + sizeof(LsmTask);
  u.upload = cv.take<char>(u.upload_bytes);
  u.bk = (DevBasket*)u.upload;
  u.ao = u.upload ? (DevOpt*)(u.upload + u.off_opts) : nullptr;
  u.task = u.upload ? (LsmTask*)(u.upload + u.off_task) : nullptr;
  u.dl = (u.upload && op == 3) ? (float*)(u.upload + u.off_dl) : nullptr;
  u.lpp = basket_lanes_per_path(d, P, num_cus);
  u.nblk = (int)((P * u.lpp + 255) / 256);  // blocks of 256 / lpp paths
  u.nchunk = (int)((P + kBasketChunk - 1) / kBasketChunk);
  u.rows = cv.take<double>((size_t)u.nblk * 2);
  u.sums = cv.take<double>((size_t)std::max(std::max(2, basket_ncol(d)), 2 * risk_cols(d)));
  if (op == 2) {
    u.rec = cv.take<float>((size_t)(1 + 2 * d) * P);
    u.part = cv.take<double>((size_t)u.nchunk * basket_ncol(d));
  }
  if (op == 3) {
    u.rec = cv.take<float>((size_t)risk_cols(d) * P);
    u.part = cv.take<double>((size_t)u.nchunk * 2 * risk_cols(d));
  }
  if (basket_american(b)) {
    u.xs = cv.take<float>((size_t)P * N);
    u.vs = cv.take<float>((size_t)P * N);
    u.tau = cv.take<int32_t>(P);
    u.gram = cv.take<float>((size_t)(N + 1) * lsm_gram_chunks(P) * kLsmGramRow10);
    u.fac = cv.take<double>((size_t)(N + 1) * kLsmFacRec10);
    u.zero_words = 16 + 2 * (int64_t)kLsmXchgWords10;
    u.zero = cv.take<uint32_t>((size_t)u.zero_words);
    u.partials = cv.take<double>((size_t)std::max((int)((P + 255) / 256), 256) * 2);
    u.beta64 = cv.take<double>((size_t)(N + 1) * SIMR_BASKET_NB);
    u.results = cv.take<double>(4);
    u.wcash = cv.take<float>((size_t)P);
    u.gpart = cv.take<float>((size_t)((P + kLsmBlock - 1) / kLsmBlock) * 16);
    u.beta32 = cv.take<float>((size_t)(N + 1) * 16);
  }
  return u;
}

size_t basket_readback_off(const BasketBufs& u) { return (u.upload_bytes + 63) / 64 * 64; }
size_t basket_pinned_bytes(const BasketBufs& u, int d) {
  return basket_readback_off(u) + sizeof(double) * (size_t)std::max(std::max(4, basket_ncol(d)), 2 * risk_cols(d));
}

// The step constants of every asset, the basket constants and (American) the induction task,
// copied to the workspace in one transfer.
simr_status basket_upload(simr_ctx* c, int scheme, const simr_basket& b, const BasketBufs& u, const LsmTask* task,
                          hipStream_t s) {
  char* up = (char*)c->pinned;
  const DevBasket k = make_devbasket(b);
  std::memcpy(up, &k, sizeof k);
  for (int i = 0; i < b.assets; ++i) {
    DevOpt o;
    simr_status st = devopt_for(c, scheme, basket_asset(b, i), &o);
    if (st != SIMR_OK) return st;
    std::memcpy(up + u.off_opts + sizeof(DevOpt) * (size_t)i, &o, sizeof o);
  }
  if (task) std::memcpy(up + u.off_task, task, sizeof(LsmTask));
  SIMR_HIP(hipMemcpyAsync(u.upload, up, u.upload_bytes, hipMemcpyHostToDevice, s));
  return SIMR_OK;
}

// The constants the Longstaff-Schwartz kernels read, for the basket's write-out: spot B_0,
// strike K, long variance thetabar = sum w_i S0_i theta_i / B_0, r dt, payoff, steps, paths.
DevOpt basket_lsm_devopt(const simr_basket& b) {
  simr_option o;
  std::memset(&o, 0, sizeof o);
  const double B0 = basket_b0(b);
  double th = 0.0;
  for (int i = 0; i < b.assets; ++i) th += b.w[i] * b.S0[i] * b.theta[i];
  o.S0 = B0;
  o.K = b.K;
  o.T = b.T;
  o.r = b.r;
  o.kappa = 1.0;
  o.theta = th / B0;
  o.payoff = b.payoff;
  o.steps = b.steps;
  o.paths = b.paths;
  return make_devopt(o);
}

double basket_intrinsic(const simr_basket& b, double B) {
  const double h = (b.payoff == SIMR_EURO_CALL || b.payoff == SIMR_AMER_CALL) ? B - b.K : b.K - B;
  return h > 0.0 ? h : 0.0;
}

// American basket by Longstaff-Schwartz: the write-out, the Gram pre-pass and the cooperative
// induction on the 10-function basis, then the finish; synchronises the stream.
simr_status basket_american_run(simr_ctx* c, int scheme, const simr_basket& b, const BasketBufs& u, bool want_beta,
                                hipStream_t s, simr_result* out) {
  std::vector<int> grids;
  std::vector<LsmLaunchSet> sets;
  if (!c->lsm_per_date) sets = lsm_coop_plan({b.paths}, c->num_cus, c->lsm_grid_max, &grids, SIMR_BASKET_NB);
  const bool coop = !sets.empty();  // else one launch per date
  LsmTask t;
  std::memset(&t, 0, sizeof t);
  t.o = basket_lsm_devopt(b);
  t.xs = u.xs;
  t.vs = u.vs;
  t.fac = u.fac;
  t.tau = u.tau;
  t.xchg = (unsigned long long*)(u.zero + 16);
  t.partials = u.partials;
  t.beta64 = want_beta ? u.beta64 : nullptr;
  t.flags = (const int32_t*)(u.zero + 1);
  t.block0 = 0;
  t.nblocks = coop ? grids[0] : (int)((b.paths + kLsmBlock - 1) / kLsmBlock);
  simr_status st = basket_upload(c, scheme, b, u, &t, s);
  if (st != SIMR_OK) return st;
  int32_t* flags = (int32_t*)(u.zero + 1);
  int32_t* status = (int32_t*)(u.zero + 2);
  {
    Prof pf(c, SIMR_PROF_SPILL, s);
    SIMR_HIP(launch_basket_paths(scheme, 2, b.assets, b.paths, u.lpp, u.bk, u.ao, nullptr, u.xs, u.vs, nullptr, u.zero,
                                 u.zero_words, nullptr, s));
  }
  if (c->lsm_fail_test && coop) SIMR_HIP(hipMemsetD32Async((hipDeviceptr_t)status, 1u, 1, s));
  {
    Prof pf(c, SIMR_PROF_GRAM, s);
    SIMR_HIP(launch_lsm_gram(t.o, u.xs, u.vs, u.gram, s, SIMR_BASKET_NB));
  }
  {
    Prof pf(c, SIMR_PROF_FACTOR, s);
    SIMR_HIP(launch_lsm_factor(t.o, b.r * b.T / b.steps, u.gram, u.fac, flags, s, SIMR_BASKET_NB));
  }
  {
    Prof pf(c, SIMR_PROF_LSM, s);
    if (coop) {
      const LsmLaunchSet& ls = sets[0];
      SIMR_HIP(launch_lsm_coop(u.task, 1, ls.block, ls.ppl, ls.grid, status, s, SIMR_BASKET_NB));
    } else {
      SIMR_HIP(launch_lsm_dates(t.o, u.xs, u.vs, u.fac, u.wcash, u.tau, u.gpart, u.beta32, t.beta64, u.zero + 3,
                                u.partials, s, SIMR_BASKET_NB));
    }
  }
  SIMR_HIP(launch_finalize_tasks(u.task, 1, status, u.results, s));
  double* rb = (double*)((char*)c->pinned + basket_readback_off(u));
  SIMR_HIP(hipMemcpyAsync(rb, u.results, sizeof(double) * 2 + sizeof(int32_t) * 2, hipMemcpyDeviceToHost, s));
  SIMR_HIP(hipStreamSynchronize(s));
  const int32_t* fl = (const int32_t*)(rb + 2);
  if (fl[1] != 0) return fail(SIMR_ENUMERIC, "Longstaff-Schwartz exchange wait timed out");
  double mean, se;
  mean_se(rb[0], rb[1], b.paths, &mean, &se);
  simr_result r;
  std::memset(&r, 0, sizeof r);
  int32_t f = fl[0];
  const double h0 = basket_intrinsic(b, basket_b0(b));
  if (h0 > mean) {
    r.price = h0;
    f |= SIMR_LSM_EXERCISE_T0;
  } else {
    r.price = mean;
    r.std_err = se;
  }
  r.paths = b.paths;
  r.lsm_flags = f;
  *out = r;
  return SIMR_OK;
}

// Common checks of the basket entry points; on success the workspace is carved.
simr_status basket_begin(simr_ctx* ctx, const simr_basket* b, const simr_params* params, int op, void* d_ws,
                         size_t ws_bytes, int* scheme, BasketBufs* u) {
  int ck;
  simr_status st = validate_params(params, scheme, &ck);
  if (st != SIMR_OK) return st;
  if ((st = validate_basket(b)) != SIMR_OK) return st;
  if (*scheme == SIMR_SCHEME_BK) return fail(SIMR_EUNSUPPORTED, "baskets do not take the Broadie-Kaya scheme");
  if (!ctx) return fail(SIMR_EINVAL, "ctx is NULL");
  Carve probe(nullptr);
  carve_basket(probe, *b, op, kWorkspaceCus);
  if (!d_ws || ws_bytes < probe.off)
    return fail(SIMR_EINVAL, "workspace too small: %zu < %zu bytes", ws_bytes, probe.off);
  Carve cv(d_ws);
  *u = carve_basket(cv, *b, op, ctx->num_cus);
  return ensure_pinned(ctx, basket_pinned_bytes(*u, b->assets));
}

// European basket: one launch (optionally writing the per-path terminal values), the block
// sums, one read-back.
simr_status basket_european_run(simr_ctx* c, int scheme, const simr_basket& b, const BasketBufs& u, float* d_xT,
                                float* d_vT, float* d_pay, hipStream_t s, simr_result* out) {
  simr_status st = basket_upload(c, scheme, b, u, nullptr, s);
  if (st != SIMR_OK) return st;
  {
    Prof pf(c, SIMR_PROF_PRICE, s);
    SIMR_HIP(launch_basket_paths(scheme, 0, b.assets, b.paths, u.lpp, u.bk, u.ao, nullptr, d_xT, d_vT, d_pay, nullptr, 0,
                                 u.rows, s));
  }
  SIMR_HIP(launch_finalize_rows(u.rows, 2, nullptr, 0, u.nblk, u.sums, s));
  double* rb = (double*)((char*)c->pinned + basket_readback_off(u));
  SIMR_HIP(hipMemcpyAsync(rb, u.sums, sizeof(double) * 2, hipMemcpyDeviceToHost, s));
  SIMR_HIP(hipStreamSynchronize(s));
  simr_result r;
  std::memset(&r, 0, sizeof r);
  mean_se(rb[0], rb[1], b.paths, &r.price, &r.std_err);
  r.paths = b.paths;
  *out = r;
  return SIMR_OK;
}

}  // namespace

extern "C" {

simr_status simr_basket_workspace_size(simr_ctx* ctx, int op, const simr_basket* b, const simr_params* params,
                                       size_t* bytes) {
  (void)ctx;
  if (!bytes) return fail(SIMR_EINVAL, "bytes is NULL");
  if (op != 0 && op != 2 && op != 3) return fail(SIMR_EINVAL, "basket op must be 0 (price), 2 (greeks) or 3 (risk)");
  int scheme, ck;
  simr_status st = validate_params(params, &scheme, &ck);
  if (st != SIMR_OK) return st;
  if ((st = validate_basket(b)) != SIMR_OK) return st;
  if (scheme == SIMR_SCHEME_BK) return fail(SIMR_EUNSUPPORTED, "baskets do not take the Broadie-Kaya scheme");
  Carve cv(nullptr);
  carve_basket(cv, *b, op, kWorkspaceCus);
  *bytes = cv.off;
  return SIMR_OK;
}

simr_status simr_basket_price(simr_ctx* ctx, const simr_basket* b, const simr_params* params, simr_result* out,
                              void* d_ws, size_t ws_bytes, void* stream) {
  if (!out) return fail(SIMR_EINVAL, "out is NULL");
  int scheme;
  BasketBufs u;
  simr_status st = basket_begin(ctx, b, params, 0, d_ws, ws_bytes, &scheme, &u);
  if (st != SIMR_OK) return st;
  DeviceGuard g(ctx);
  hipStream_t s = (hipStream_t)stream;
  if (basket_american(*b)) return basket_american_run(ctx, scheme, *b, u, false, s, out);
  return basket_european_run(ctx, scheme, *b, u, nullptr, nullptr, nullptr, s, out);
}

simr_status simr_basket_greeks(simr_ctx* ctx, const simr_basket* b, const simr_params* params,
                               simr_basket_greeks_result* out, void* d_ws, size_t ws_bytes, void* stream) {
  if (!out) return fail(SIMR_EINVAL, "out is NULL");
  int scheme;
  BasketBufs u;
  simr_status st = basket_begin(ctx, b, params, 2, d_ws, ws_bytes, &scheme, &u);
  if (st != SIMR_OK) return st;
  DeviceGuard g(ctx);
  hipStream_t s = (hipStream_t)stream;
  const int d = b->assets;
  const double nan = std::nan("");
  simr_basket_greeks_result r;
  std::memset(&r, 0, sizeof r);
  const bool am = basket_american(*b);
  if (am) {
    simr_result lr;
    if ((st = basket_american_run(ctx, scheme, *b, u, false, s, &lr)) != SIMR_OK) return st;
    r.price = lr.price;
    r.std_err = lr.std_err;
    r.lsm_flags = lr.lsm_flags;
    for (int i = 0; i < d; ++i)
      for (int j = 0; j < d; ++j) {
        r.gamma[i * SIMR_MAX_ASSETS + j] = nan;
        r.gamma_se[i * SIMR_MAX_ASSETS + j] = nan;
      }
    if (lr.lsm_flags & SIMR_LSM_EXERCISE_T0) {  // h(B_0): delta_i = h'(B_0) w_i
      const double sgn = b->payoff == SIMR_AMER_CALL ? 1.0 : -1.0;
      for (int i = 0; i < d; ++i) r.delta[i] = sgn * b->w[i];
      *out = r;
      return SIMR_OK;
    }
  } else {
    if ((st = basket_upload(ctx, scheme, *b, u, nullptr, s)) != SIMR_OK) return st;
  }
  const int ncol = am ? 2 + 2 * d : basket_ncol(d);
  {
    Prof pf(ctx, SIMR_PROF_PRICE, s);
    SIMR_HIP(launch_basket_paths(scheme, 1, d, b->paths, u.lpp, u.bk, u.ao, am ? u.tau : nullptr, u.rec, nullptr, nullptr,
                                 nullptr, 0, nullptr, s));
  }
  SIMR_HIP(launch_basket_moments(u.bk, b->paths, u.rec, ncol, u.part, s));
  SIMR_HIP(launch_finalize_rows(u.part, ncol, nullptr, 0, u.nchunk, u.sums, s));
  double* rb = (double*)((char*)ctx->pinned + basket_readback_off(u));
  SIMR_HIP(hipMemcpyAsync(rb, u.sums, sizeof(double) * (size_t)ncol, hipMemcpyDeviceToHost, s));
  SIMR_HIP(hipStreamSynchronize(s));
  const int64_t P = b->paths;
  if (!am) mean_se(rb[0], rb[1], P, &r.price, &r.std_err);
  for (int i = 0; i < d; ++i) mean_se(rb[2 + i], rb[2 + d + i], P, &r.delta[i], &r.delta_se[i]);
  if (!am) {
    int q = 0;
    for (int i = 0; i < d; ++i)
      for (int j = i; j < d; ++j, ++q) {
        double m, se;
        mean_se(rb[2 + 2 * d + 2 * q], rb[2 + 2 * d + 2 * q + 1], P, &m, &se);
        r.gamma[i * SIMR_MAX_ASSETS + j] = r.gamma[j * SIMR_MAX_ASSETS + i] = m;
        r.gamma_se[i * SIMR_MAX_ASSETS + j] = r.gamma_se[j * SIMR_MAX_ASSETS + i] = se;
      }
  }
  *out = r;
  return SIMR_OK;
}

simr_status simr_basket_risk(simr_ctx* ctx, const simr_basket* b, const simr_params* params,
                             simr_basket_risk_result* out, void* d_ws, size_t ws_bytes, void* stream) {
  if (!out) return fail(SIMR_EINVAL, "out is NULL");
  int sch, ck;
  simr_status st = validate_params(params, &sch, &ck);
  if (st != SIMR_OK) return st;
  if ((st = validate_basket(b)) != SIMR_OK) return st;
  if (b->assets > kRiskMaxAssets)
    return fail(SIMR_EUNSUPPORTED, "basket risk Greeks take at most %d assets (got %d)", kRiskMaxAssets, b->assets);
  if (sch != SIMR_SCHEME_QE && sch != SIMR_SCHEME_FTE && sch != SIMR_SCHEME_TG)
    return fail(SIMR_EUNSUPPORTED, "basket risk Greeks take the QE, full-truncation Euler and truncated Gaussian "
                                   "schemes");
  int scheme;
  BasketBufs u;
  if ((st = basket_begin(ctx, b, params, 3, d_ws, ws_bytes, &scheme, &u)) != SIMR_OK) return st;
  DeviceGuard g(ctx);
  hipStream_t s = (hipStream_t)stream;
  const int d = b->assets;
  // the Cholesky factor's derivative of every pair, into the upload region of the staging
  std::vector<double> L;
  if (!corr_factor(*b, &L)) return fail(SIMR_EINVAL, "basket corr is not positive definite");
  float* dlh = (float*)((char*)ctx->pinned + u.off_dl);
  std::memset(dlh, 0, sizeof(float) * (size_t)kRiskPairs * kRiskTri);
  std::vector<double> dL((size_t)d * d);
  for (int i = 1; i < d; ++i)
    for (int j = 0; j < i; ++j) {
      chol_derivative(d, L, i, j, dL.data());
      float* dq = dlh + (size_t)(i * (i - 1) / 2 + j) * kRiskTri;
      for (int r = 0; r < d; ++r)
        for (int c = 0; c <= r; ++c) dq[r * (r + 1) / 2 + c] = (float)dL[r * d + c];
    }
  simr_basket_risk_result r;
  std::memset(&r, 0, sizeof r);
  const bool am = basket_american(*b);
  if (am) {  // the Longstaff-Schwartz pass (its upload carries the derivatives), then its policy fixed
    simr_result lr;
    if ((st = basket_american_run(ctx, scheme, *b, u, false, s, &lr)) != SIMR_OK) return st;
    r.price = lr.price;
    r.std_err = lr.std_err;
    r.lsm_flags = lr.lsm_flags;
    if (lr.lsm_flags & SIMR_LSM_EXERCISE_T0) {  // h(B_0) moves with no model parameter
      *out = r;
      return SIMR_OK;
    }
  } else {
    if ((st = basket_upload(ctx, scheme, *b, u, nullptr, s)) != SIMR_OK) return st;
  }
  const int nrec = risk_cols(d);
  {
    Prof pf(ctx, SIMR_PROF_PRICE, s);
    SIMR_HIP(launch_basket_risk(scheme, d, b->paths, u.bk, u.ao, am ? u.tau : nullptr, u.rec, u.dl, s));
  }
  SIMR_HIP(launch_record_moments(u.rec, nrec, b->paths, u.part, s));
  SIMR_HIP(launch_finalize_rows(u.part, 2 * nrec, nullptr, 0, u.nchunk, u.sums, s));
  double* rb = (double*)((char*)ctx->pinned + basket_readback_off(u));
  SIMR_HIP(hipMemcpyAsync(rb, u.sums, sizeof(double) * 2 * (size_t)nrec, hipMemcpyDeviceToHost, s));
  SIMR_HIP(hipStreamSynchronize(s));
  const int64_t P = b->paths;
  if (!am) mean_se(rb[0], rb[1], P, &r.price, &r.std_err);
  for (int i = 0; i < d; ++i) {
    mean_se(rb[2 * (1 + i)], rb[2 * (1 + i) + 1], P, &r.vega_v0[i], &r.vega_v0_se[i]);
    mean_se(rb[2 * (1 + d + i)], rb[2 * (1 + d + i) + 1], P, &r.vega_theta[i], &r.vega_theta_se[i]);
  }
  for (int i = 1; i < d; ++i)
    for (int j = 0; j < i; ++j) {
      const int c = 1 + 2 * d + i * (i - 1) / 2 + j;
      double m, se;
      mean_se(rb[2 * c], rb[2 * c + 1], P, &m, &se);
      r.dcorr[i * SIMR_MAX_ASSETS + j] = r.dcorr[j * SIMR_MAX_ASSETS + i] = m;
      r.dcorr_se[i * SIMR_MAX_ASSETS + j] = r.dcorr_se[j * SIMR_MAX_ASSETS + i] = se;
    }
  *out = r;
  return SIMR_OK;
}

simr_status simr_debug_basket_paths(simr_ctx* ctx, const simr_basket* b, const simr_params* params, float* d_xT,
                                    float* d_vT, float* d_payoff, void* d_ws, size_t ws_bytes, void* stream) {
  int scheme;
  BasketBufs u;
  simr_status st = basket_begin(ctx, b, params, 0, d_ws, ws_bytes, &scheme, &u);
  if (st != SIMR_OK) return st;
  DeviceGuard g(ctx);
  simr_result r;
  return basket_european_run(ctx, scheme, *b, u, d_xT, d_vT, d_payoff, (hipStream_t)stream, &r);
}

simr_status simr_debug_basket_lsm(simr_ctx* ctx, const simr_basket* b, const simr_params* params, simr_result* out,
                                  int32_t* d_tau, double* d_beta, void* d_ws, size_t ws_bytes, void* stream) {
  if (!out) return fail(SIMR_EINVAL, "out is NULL");
  if (b && !basket_american(*b)) return fail(SIMR_EINVAL, "simr_debug_basket_lsm needs an American basket");
  int scheme;
  BasketBufs u;
  simr_status st = basket_begin(ctx, b, params, 0, d_ws, ws_bytes, &scheme, &u);
  if (st != SIMR_OK) return st;
  DeviceGuard g(ctx);
  hipStream_t s = (hipStream_t)stream;
  const size_t nbeta = sizeof(double) * SIMR_BASKET_NB * (size_t)(b->steps + 1);
  SIMR_HIP(hipMemsetAsync(u.beta64, 0, nbeta, s));  // dates with no regression keep zero coefficients
  if ((st = basket_american_run(ctx, scheme, *b, u, true, s, out)) != SIMR_OK) return st;
  if (d_tau) SIMR_HIP(hipMemcpyAsync(d_tau, u.tau, sizeof(int32_t) * (size_t)b->paths, hipMemcpyDeviceToDevice, s));
  if (d_beta) SIMR_HIP(hipMemcpyAsync(d_beta, u.beta64, nbeta, hipMemcpyDeviceToDevice, s));
  SIMR_HIP(hipStreamSynchronize(s));
  return SIMR_OK;
}

}  // extern "C"
