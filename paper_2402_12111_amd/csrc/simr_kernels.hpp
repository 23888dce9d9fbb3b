// simr_kernels.hpp -- launch interface between the host runtime and the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "simr_device.hpp"

namespace simr {

constexpr int kLsmBlock = 256;  // block of the Longstaff-Schwartz kernels (one path per lane)
// Block of the adjoint kernel (one path per lane, ordered within the block): the largest of
// 1024, 512, 256 threads that still gives every CU a block (larger blocks order more paths
// together); at most 512 for 32-step segments and for the extended Greeks, whose registers need
// the larger per-thread budget.
inline int adjoint_block(int64_t paths, int ck, bool ext, int num_cus) {
  for (int b = (ck >= 32 || ext) ? 512 : 1024; b > 256; b /= 2)
    if ((paths + b - 1) / b >= num_cus) return b;
  return 256;
}
constexpr int kAdjMinBlock = 256;
constexpr int kCkBlock = 256;    // block of the checkpointing forward pass
constexpr int kAdjClasses = 64;  // exercise-index classes the adjoint orders its paths by

// European batch launch: persistent grid over an atomic unit queue.
struct BatchLaunch {
  const DevOpt* opts;
  const int32_t* order;    // option indices by descending cost
  const int32_t* uprefix;  // unit prefix sums over `order`, nopt + 1 entries
  int32_t nopt, nunits;
  uint32_t* counter;       // queue head, zero before the launch
  double* partials;        // {sum X, sum X^2} per (option, tile) slot
  int grid, block, ppl;
};

// Device state of one Longstaff-Schwartz backward induction.
struct LsmState {
  float* gpart;      // per-block FP32 regression sums, 32 floats per block
  uint32_t* ticket;  // blocks finished with the current date (reset by the last one)
  int32_t* flags;    // SIMR_LSM_FEW_ITM | SIMR_LSM_DROPPED
  float* beta32;     // per date: 6 coefficients (FP32), [6] = 1 if a regression ran
  double* beta64;    // per date: the 6 FP64 coefficients
};

// One American option of a cooperative backward-induction launch: blocks [block0, block0 +
// nblocks) of the launch work on it and exchange only among themselves.
struct LsmTask {
  DevOpt o;
  const float* xs;           // spilled states, row n - 1 = date n, P floats per row
  const float* vs;
  const double* fac;         // factor record of every date
  int32_t* tau;              // out: exercise index per path
  unsigned long long* xchg;  // [2][nblocks][8] tagged words of the blocks' sums; zero before the launch
  double* partials;          // out: {sum X, sum X^2} per block of the task
  double* beta64;            // out, may be null: the 6 FP64 coefficients per date (first block)
  const int32_t* flags;      // SIMR_LSM_FEW_ITM | SIMR_LSM_DROPPED of the option (read by the finish)
  int32_t block0, nblocks;
};

// Chunks of paths per date of the Gram pre-pass: each lane sums at most 16 paths in FP32.
inline int lsm_gram_chunks(int64_t paths) {
  return (int)((paths + (int64_t)kLsmBlock * 16 - 1) / ((int64_t)kLsmBlock * 16));
}
constexpr int kLsmGramRow = 16;  // floats per (date, chunk) row of Gram sums (15 moments)
constexpr int kLsmFacRec = 64;   // doubles per date of factor record
constexpr int kLsmXchgWords = 2 * 256 * 8;  // 64-bit exchange words of the cooperative induction
// The same for the basket regression on 10 functions (55 Gram entries and the count per row,
// M of 100 entries per record, 16 exchange words per block and date).
constexpr int kLsmGramRow10 = 56;
constexpr int kLsmFacRec10 = 128;
constexpr int kLsmXchgWords10 = 2 * 256 * 16;

// Cooperative launches of a list of American options: consecutive tasks [first, first + count)
// share one launch of `block` threads x `ppl` paths per lane.
struct LsmLaunchSet { int first, count, block, ppl, grid; };
// Splits options with the given path counts into launch sets whose blocks are co-resident, each
// option taking ceil(P / (1024 ppl)) blocks of the paths per block it would take alone (at most
// `gmax` blocks if possible, else 256), run as 1024 threads x ppl or 256 threads x 4 ppl (the
// same bits).  Returns the sets; empty if some option fits no shape.  grids[i] receives option
// i's blocks.  nb: functions of the regression basis (6, or 10 for baskets: 1024-thread blocks
// only).  block: 0 lets each set take the block size that holds more of its options; 1024 or
// 256 restricts every set to that size.
std::vector<LsmLaunchSet> lsm_coop_plan(const std::vector<int64_t>& paths, int num_cus, int gmax,
                                        std::vector<int>* grids, int nb = 6, int block = 0);
// The Gram and right-hand-side sums of every date, then (launch_lsm_factor, same stream) their
// FP64 factorisations; rdt = r T / N in FP64 (the factor records carry e^{r n dt}).
hipError_t launch_lsm_gram(const DevOpt& o, const float* xs, const float* vs, float* gram, hipStream_t s,
                           int nb = 6);
hipError_t launch_lsm_factor(const DevOpt& o, double rdt, const float* gram, double* fac, int32_t* flags,
                             hipStream_t s, int nb = 6);
// tasks: device array, sorted by block0, block0 relative to this launch.
hipError_t launch_lsm_coop(const LsmTask* tasks, int ntasks, int block, int ppl, int grid, int32_t* status,
                           hipStream_t s, int nb = 6);
// out[2 t], out[2 t + 1] = sums of task t's block partials in block order (FP64); then, as int32
// after the 2 ntasks doubles: the flags of every task, then *status.
hipError_t launch_finalize_tasks(const LsmTask* tasks, int ntasks, const int32_t* status, double* out,
                                 hipStream_t s);
// The induction with one launch per date on the factor records (paths beyond the cooperative
// capacity), then the finish rows in `partials` (one pair per block of kLsmBlock paths).  wcash:
// P floats; gpart: ceil(P / kLsmBlock) * kXW floats; beta32: (N + 1) * kXW floats; ticket: one
// zeroed word.  Basis of nb = 10 functions.
hipError_t launch_lsm_dates(const DevOpt& o, const float* xs, const float* vs, const double* fac, float* wcash,
                            int32_t* tau, float* gpart, float* beta32, double* beta64, uint32_t* ticket,
                            double* partials, hipStream_t s, int nb);

hipError_t launch_batch_price(int scheme, const BatchLaunch& L, hipStream_t s);
int batch_kernel_occupancy(int scheme, int block, int ppl);
hipError_t launch_finalize_rows(const double* rows, int ncol, const DevOpt* opts, int nopt, int nrows, double* out,
                                hipStream_t s);
hipError_t launch_reset_words(uint32_t* p, int64_t n, hipStream_t s);
// Copies `bytes` (a multiple of 4, at most 1024) of host memory to device memory `dst` through a
// kernel argument: no host staging buffer, no copy engine.
hipError_t launch_stage_record(const void* src, size_t bytes, void* dst, hipStream_t s);
// Also zeroes zero[0, nzero) (may be null with nzero = 0).
hipError_t launch_forward_spill(int scheme, const DevOpt& o, float* xs, float* vs, uint32_t* zero, int64_t nzero,
                                hipStream_t s);
hipError_t launch_lsm(const DevOpt& o, const float* xs, const float* vs, float* hcash, int32_t* tau,
                      const LsmState& st, double* partials, hipStream_t s);
hipError_t launch_forward_ckpt(int scheme, const DevOpt& o, int ck, float* ckbuf, float* xN, double* partials,
                               hipStream_t s);
// gpart: 14 (ext: 18) doubles per block of `block` paths (adjoint_block).
hipError_t launch_adjoint(int scheme, const DevOpt& o, int ck, int block, bool ext, const float* ck_base,
                          size_t ck_stride, const float* xstop, const int32_t* tau, double* gpart, hipStream_t s);
hipError_t launch_debug_draws(uint64_t seed, uint32_t stream, int64_t path0, int64_t npaths, int32_t step0,
                              int32_t nsteps, uint32_t* words, float* unif, float* norm, hipStream_t s);
hipError_t launch_debug_paths(int scheme, const DevOpt& o, float* xT, float* vT, float* pay, hipStream_t s);

// ---------------------------------------------------------------------------------------------
// Correlated baskets.
// ---------------------------------------------------------------------------------------------
constexpr int kMaxAssets = 32;
constexpr int kBasketTri = kMaxAssets * (kMaxAssets + 1) / 2;
constexpr int kBasketChunk = 128;  // paths per block of the Greeks moments
// Basket risk Greeks (vegas, correlation sensitivities): at most 8 assets; the derivative of the
// Cholesky factor of each pair is packed by rows like L, kRiskTri floats per pair.
constexpr int kRiskMaxAssets = 8;
constexpr int kRiskTri = kRiskMaxAssets * (kRiskMaxAssets + 1) / 2;
constexpr int kRiskPairs = kRiskMaxAssets * (kRiskMaxAssets - 1) / 2;
constexpr int kRiskRecCols = 1 + 2 * kRiskMaxAssets + kRiskPairs;  // risk record columns at most

// Basket-level constants (FP64 on the host, rounded once); the per-asset step constants are a
// DevOpt per asset.
struct DevBasket {
  int32_t d, steps, paths, payoff;
  uint32_t stream, seed_lo, seed_hi;
  int32_t pad;
  float K, disc, rdt, invB0;   // strike, e^{-rT}, r dt, 1 / B_0
  float w[kMaxAssets];         // weights
  float wS0[kMaxAssets];       // w_i S0_i
  float S0[kMaxAssets];
  float L[kBasketTri];         // lower Cholesky factor of C by rows: L_ik at i (i + 1) / 2 + k
  float Linv[kBasketTri];      // L^{-1}, the same packing
};

// The smallest compiled asset tile (4, 8, 16, 32) holding d assets.
int basket_tier(int d);
// Lanes per path of the basket kernels: 1 (one path per lane), or 4 (the split kernel) for more
// than 8 assets and fewer than two waves per SIMD at one path per lane.
int basket_lanes_per_path(int d, int64_t paths, int num_cus);
// mode 0 price, 1 Greeks records, 2 Longstaff-Schwartz write-out (see basket_path_kernel);
// lpp from basket_lanes_per_path (rows: 2 doubles per block of 256 / lpp paths).
hipError_t launch_basket_paths(int scheme, int mode, int d, int64_t paths, int lpp, const DevBasket* bk,
                               const DevOpt* ao, const int32_t* tau, float* o1, float* o2, float* o3, uint32_t* zero,
                               int64_t nzero, double* rows, hipStream_t s);
// Risk records of a basket of d <= kRiskMaxAssets assets (QE, full-truncation Euler or truncated
// Gaussian; see basket_path_kernel MODE 3): 1 + 2 d + d (d - 1) / 2 columns of P floats at rec;
// dl holds the Cholesky factor's derivative of each pair, kRiskTri floats per pair.
hipError_t launch_basket_risk(int scheme, int d, int64_t paths, const DevBasket* bk, const DevOpt* ao,
                              const int32_t* tau, float* rec, const float* dl, hipStream_t s);
// Per chunk of kBasketChunk paths, FP64 sums and sums of squares of ncol record columns:
// ceil(P / kBasketChunk) rows of 2 ncol doubles.
hipError_t launch_record_moments(const float* rec, int ncol, int64_t paths, double* part, hipStream_t s);
// Per-chunk FP64 moments of the Greeks records: ceil(P / kBasketChunk) rows of ncol doubles.
hipError_t launch_basket_moments(const DevBasket* bk, int64_t paths, const float* rec, int ncol, double* part,
                                 hipStream_t s);

}  // namespace simr
