// simr_kernels.hpp -- launch interface between the host runtime and the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "simr_device.hpp"

namespace simr {

constexpr int kLsmBlock = 256;  // block of the Longstaff-Schwartz kernels (one path per lane)
constexpr int kAdjBlock = 256;  // block of the Greeks kernels (one path per lane)

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

// Device state of the persistent (cooperative) backward induction.
struct LsmCoop {
  unsigned long long* xchg;  // [2][G][8] tagged words of the blocks' sums; zero before the launch
  int32_t* status;           // nonzero if a wait timed out
  int32_t* flags;    // SIMR_LSM_FEW_ITM | SIMR_LSM_DROPPED
  double* beta64;    // per date: the 6 FP64 coefficients (written by block 0)
};

// Chunks of paths per date of the Gram pre-pass: each lane sums at most 8 paths in FP32.
inline int lsm_gram_chunks(int64_t paths) {
  return (int)((paths + (int64_t)kLsmBlock * 8 - 1) / ((int64_t)kLsmBlock * 8));
}
constexpr int kLsmGramRow = 24;  // floats per (date, chunk) row of Gram sums
constexpr int kLsmFacRec = 64;   // doubles per date of factor record
constexpr int kLsmXchgWords = 2 * 256 * 8;  // 64-bit exchange words of the cooperative induction

int lsm_coop_plan(int64_t paths, int num_cus, int gmax, int* grid_out, int* block_out);
hipError_t launch_lsm_gram(const DevOpt& o, const float* xs, const float* vs, float* gram, double* fac,
                           int32_t* flags, hipStream_t s);
hipError_t launch_lsm_coop(const DevOpt& o, int block, int ppl, int grid, const float* xs, const float* vs,
                           const double* fac, float* hcash, int32_t* tau, const LsmCoop& st, double* partials,
                           hipStream_t s);

hipError_t launch_batch_price(int scheme, const BatchLaunch& L, hipStream_t s);
int batch_kernel_occupancy(int scheme, int block, int ppl);
hipError_t launch_finalize_rows(const double* rows, int ncol, const DevOpt* opts, int nopt, int nrows, double* out,
                                hipStream_t s);
hipError_t launch_reset_words(uint32_t* p, int n, hipStream_t s);
hipError_t launch_forward_spill(int scheme, const DevOpt& o, float* xs, float* vs, hipStream_t s);
hipError_t launch_lsm(const DevOpt& o, const float* xs, const float* vs, float* hcash, int32_t* tau,
                      const LsmState& st, double* partials, hipStream_t s);
hipError_t launch_forward_ckpt(const DevOpt& o, int ck, float* ckbuf, float* xN, double* partials, hipStream_t s);
hipError_t launch_adjoint(const DevOpt& o, int ck, const float* ck_base, size_t ck_stride, const float* xstop,
                          const int32_t* tau, double* gpart, hipStream_t s);
hipError_t launch_debug_draws(uint64_t seed, uint32_t stream, int64_t path0, int64_t npaths, int32_t step0,
                              int32_t nsteps, uint32_t* words, float* unif, float* norm, hipStream_t s);
hipError_t launch_debug_paths(int scheme, const DevOpt& o, float* xT, float* vT, float* pay, hipStream_t s);

}  // namespace simr
