// simr_kernels.hip -- gfx950 kernels of the Heston Monte Carlo / Longstaff-Schwartz hot path.
//
// Mapping of the paper's SIMR dataflow stages (Sec. 5, opening paragraph) onto the GPU: the
// stages VariancePathQE -> LogPricePathQE -> AssetPathExponential run fused in registers, one
// path per lane, time sequential per lane (the loop-carried state the paper keeps in a cached
// buffer, Listing 2, and feeds back through its loopback adaptor, Sec. 5.1, lives in VGPRs);
// writeLongstaffSchwartzPath is the coalesced spill of (x, v) per date; and
// longstaffSchwartzPathReduction is the per-date regression reduction: wave64 shuffles, an
// LDS tree, FP64 cross-block sums and an FP64 solve in the last block to finish.
#include <algorithm>
#include <cstring>

#include "simr_device.hpp"
#include "simr_kernels.hpp"

namespace simr {

// ---------------------------------------------------------------------------------------------
// European pricing: persistent kernel over (option, path-tile) units from an atomic queue.
// Unit u of the queue belongs to option order[i] with uprefix[i] <= u < uprefix[i + 1]
// (options sorted by descending cost, so the longest units start first).  A tile holds
// BLOCK * PPL paths: lane l, slot j takes path tile * BLOCK * PPL + j * BLOCK + l.
// ---------------------------------------------------------------------------------------------
template <int SCHEME, int BLOCK, int PPL>
__global__ __launch_bounds__(BLOCK) void batch_price_kernel(const DevOpt* __restrict__ opts,
                                                            const int32_t* __restrict__ order,
                                                            const int32_t* __restrict__ uprefix,
                                                            int32_t nopt, int32_t nunits,
                                                            uint32_t* __restrict__ counter,
                                                            double* __restrict__ partials) {
  __shared__ int32_t s_unit;
  __shared__ double s_red[2 * (BLOCK / kWave)];
  for (;;) {
    __syncthreads();
    if (threadIdx.x == 0) s_unit = (int32_t)atomicAdd(counter, 1u);
    __syncthreads();
    const int32_t u = __builtin_amdgcn_readfirstlane(s_unit);
    if (u >= nunits) break;  // every block leaves once the queue is drained
    int32_t lo = 0, hi = nopt - 1;  // last i with uprefix[i] <= u
    while (lo < hi) {
      const int32_t mid = (lo + hi + 1) >> 1;
      if (uprefix[mid] <= u) lo = mid; else hi = mid - 1;
    }
    const int32_t oi = __builtin_amdgcn_readfirstlane(order[lo]);
    const int32_t tile = u - uprefix[lo];
    const DevOpt o = opts[oi];
    const uint32_t base = (uint32_t)tile * (BLOCK * PPL) + threadIdx.x;

    float x[PPL], v[PPL];
#pragma unroll
    for (int j = 0; j < PPL; ++j) { x[j] = 0.0f; v[j] = o.v0; }
    for (int32_t n = 0; n < o.steps; ++n) {
#pragma unroll
      for (int j = 0; j < PPL; ++j) {
        const Draw d = draw(o, (uint32_t)n, base + j * BLOCK);
        transition<SCHEME>(o, x[j], v[j], d);
      }
    }
    Kahan k1, k2;
#pragma unroll
    for (int j = 0; j < PPL; ++j) {
      if (base + j * BLOCK < (uint32_t)o.paths) {
        const float X = o.disc * intrinsic(o, asset(o, x[j]));
        k1.add(X);
        k2.add(X * X);
      }
    }
    double vals[2] = {k1.value(), k2.value()};
    block_sum<BLOCK, 2, double>(vals, s_red);
    if (threadIdx.x == 0) {
      partials[2 * (size_t)(o.slot0 + tile)] = vals[0];
      partials[2 * (size_t)(o.slot0 + tile) + 1] = vals[1];
    }
  }
}

// Sums, for each option of `opts` (one block each), its rows [slot0, slot0 + ntiles) of a
// row-major table of `ncol` doubles in a fixed order: thread t adds rows t, t + 256, ...
// sequentially, then the 256 partial sums are combined by a fixed tree.  With opts == nullptr
// a single set of rows [0, nrows) is summed, one block per column (the same order).
__global__ __launch_bounds__(256) void finalize_rows_kernel(const double* __restrict__ rows, int32_t ncol,
                                                            const DevOpt* __restrict__ opts, int32_t nrows,
                                                            double* __restrict__ out) {
  __shared__ double s[256];
  const int32_t r0 = opts ? opts[blockIdx.x].slot0 : 0;
  const int32_t nr = opts ? opts[blockIdx.x].ntiles : nrows;
  const int32_t c_begin = opts ? 0 : (int32_t)blockIdx.x;
  const int32_t c_end = opts ? ncol : (int32_t)blockIdx.x + 1;
  const size_t ob = opts ? (size_t)blockIdx.x * ncol : 0;
  for (int32_t c = c_begin; c < c_end; ++c) {
    double acc = 0.0;
    for (int32_t r = threadIdx.x; r < nr; r += 256) acc += rows[(size_t)(r0 + r) * ncol + c];
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
      if ((int)threadIdx.x < w) s[threadIdx.x] += s[threadIdx.x + w];
      __syncthreads();
    }
    if (threadIdx.x == 0) out[ob + c] = s[0];
    __syncthreads();
  }
}

// Copies a small host record (passed by value as the kernel argument) into device memory: the
// allocation-free entry point stages its option record this way, with no host staging buffer.
struct Record1K {
  uint32_t w[256];
};

__global__ __launch_bounds__(256) void stage_record_kernel(Record1K r, uint32_t nwords, uint32_t* __restrict__ dst) {
  for (uint32_t i = threadIdx.x; i < nwords; i += 256) dst[i] = r.w[i];
}

__global__ void reset_words_kernel(uint32_t* p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0u;
}

// ---------------------------------------------------------------------------------------------
// Forward pass that writes the path states out (writeLongstaffSchwartzPath): x_n, v_n for
// n = 1..N in SoA rows of P floats (row n - 1), coalesced per wave.
// ---------------------------------------------------------------------------------------------
// A row address every lane holds the same value of, as a scalar value the compiler cannot split
// up: an access at it plus a lane's 32-bit offset then takes the scalar-base form.
__device__ __forceinline__ SIMR_GLOBAL char* uniform_row(float* row) {
  const uint64_t a = (uint64_t)(uintptr_t)row;
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)a);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(a >> 32));
  return (SIMR_GLOBAL char*)(uintptr_t)(((uint64_t)hi << 32) | lo);
}

template <int SCHEME, int BLOCK>
__global__ __launch_bounds__(BLOCK) void forward_spill_kernel(DevOpt o, float* __restrict__ xs,
                                                              float* __restrict__ vs, uint32_t* __restrict__ zero,
                                                              int64_t nzero) {
  const uint32_t p = blockIdx.x * BLOCK + threadIdx.x;
  // the words the later kernels of this option expect at zero (flags, exchange) are cleared here
  for (int64_t i = p; i < nzero; i += (int64_t)gridDim.x * BLOCK) zero[i] = 0u;
  if (p >= (uint32_t)o.paths) return;
  const size_t P = (size_t)o.paths;
  // each store at the row's uniform base plus the lane's 32-bit byte offset (paths <= 2^30):
  // the scalar-base form, with no 64-bit address arithmetic per store in the step loop
  // (otherwise the compiler adds the row offset to the lane's offset first and forms both
  // addresses with 64-bit vector adds)
  uint32_t boff = p * (uint32_t)sizeof(float);
  float x = 0.0f, v = o.v0;
  for (int32_t n = 0; n < o.steps; ++n) {
    const Draw d = draw(o, (uint32_t)n, p);
    transition<SCHEME>(o, x, v, d);
    SIMR_GLOBAL char* xr = uniform_row(xs + (size_t)n * P);
    SIMR_GLOBAL char* vr = uniform_row(vs + (size_t)n * P);
    asm volatile("" : "+v"(boff));  // a 32-bit value of this step, not a hoisted 64-bit one
    *(SIMR_GLOBAL float*)(xr + boff) = x;
    *(SIMR_GLOBAL float*)(vr + boff) = v;
  }
}

// ---------------------------------------------------------------------------------------------
// Longstaff-Schwartz backward induction.
// ---------------------------------------------------------------------------------------------

// Regression basis (1, a, a^2, c, a c, c^2), a = S/K - 1, c = v+/theta - 1: the span of
// {1, S, S^2, v, S v, v^2}, shifted and scaled so the FP32 normal equations stay well
// conditioned.  The coordinates a = (S - K) / K and c = (max(v, 0) - theta) / theta are formed
// once; the functions from them.
__device__ __forceinline__ float lsm_a(const DevOpt& o, float S) { return (S - o.K) * o.invK; }
__device__ __forceinline__ float lsm_c(const DevOpt& o, float v) { return (fmaxf(v, 0.0f) - o.theta) * o.invTheta; }

// Element at byte offset boff of the FP32 row starting at a + row0: the row base is uniform and
// the offset a 32-bit lane value, so the load takes the scalar-base, vector-offset form.
__device__ __forceinline__ float spill_at(const SIMR_GLOBAL float* __restrict__ a, size_t row0, uint32_t boff) {
  return *(const SIMR_GLOBAL float*)((const SIMR_GLOBAL char*)(a + row0) + boff);
}

__device__ __forceinline__ void lsm_basis_ac(float a, float c, float (&phi)[6]) {
  phi[0] = 1.0f;
  phi[1] = a;
  phi[2] = a * a;
  phi[3] = c;
  phi[4] = a * c;
  phi[5] = c * c;
}

__device__ __forceinline__ void lsm_basis(const DevOpt& o, float S, float v, float (&phi)[6]) {
  lsm_basis_ac(lsm_a(o, S), lsm_c(o, v), phi);
}

// Basket regression basis: the full cubic in (a, c) -- the six functions above, then a^3, a^2 c,
// a c^2, c^3 -- for NB = 10; the basis above for NB = 6.
template <int NB>
__device__ __forceinline__ void lsm_basis_nb_ac(float a, float c, float (&phi)[NB]) {
  if constexpr (NB == 6) {
    lsm_basis_ac(a, c, phi);
  } else {
    static_assert(NB == 10, "a basis of 6 or 10 functions");
    phi[0] = 1.0f;
    phi[1] = a;
    phi[2] = a * a;
    phi[3] = c;
    phi[4] = a * c;
    phi[5] = c * c;
    phi[6] = phi[2] * a;
    phi[7] = phi[2] * c;
    phi[8] = phi[4] * c;
    phi[9] = phi[5] * c;
  }
}

template <int NB>
__device__ __forceinline__ void lsm_basis_nb(const DevOpt& o, float S, float v, float (&phi)[NB]) {
  lsm_basis_nb_ac<NB>(lsm_a(o, S), lsm_c(o, v), phi);
}

// Buffer layout of the Longstaff-Schwartz kernels for a basis of NB functions.
template <int NB>
struct LsmLayout {
  // floats a (date, chunk) row of the Gram pre-pass sums: for 6 functions the 15 moments
  // sum a^p c^q, p + q <= 4 (the count first), from which every Gram entry follows; for 10 the
  // upper triangle, then the in-the-money count
  static constexpr int kSums = NB == 6 ? 15 : NB * (NB + 1) / 2 + 1;
  static constexpr int kRow = NB == 6 ? kLsmGramRow : kLsmGramRow10;  // floats per (date, chunk) row
  static constexpr int kRec = NB == 6 ? kLsmFacRec : kLsmFacRec10;    // doubles per date of factor record
  static constexpr int kRank = NB == 6 ? 48 : NB * NB;  // after M: rank, count, valid, e^{r n dt}
  static constexpr int kXW = NB <= 8 ? 8 : 16;          // exchange words per block and date
  static_assert(kSums <= kRow && kRank + 4 <= kRec && NB <= kXW, "layout");
};

// e^{-r k dt} for k dates of discounting.
__device__ __forceinline__ float discount(const DevOpt& o, int32_t k) {
  return __builtin_amdgcn_exp2f(-o.rdt * 1.44269504088896340736f * (float)k);
}

// Cash flow of every path at maturity.
template <int BLOCK>
__global__ __launch_bounds__(BLOCK) void lsm_init_kernel(DevOpt o, const float* __restrict__ xs,
                                                         float* __restrict__ hcash, int32_t* __restrict__ tau) {
  const uint32_t p = blockIdx.x * BLOCK + threadIdx.x;
  if (p >= (uint32_t)o.paths) return;
  const size_t P = (size_t)o.paths;
  hcash[p] = intrinsic(o, asset(o, xs[(size_t)(o.steps - 1) * P + p]));
  tau[p] = o.steps;
}

// Pivoted Cholesky least squares on the 6x6 normal equations in FP64: the pivot is the largest
// remaining diagonal of the Schur complement (lowest index on ties); once it is <= 1e-12 times
// the largest original diagonal the remaining columns are dropped (coefficient 0).
__device__ int solve_normal6(double (&A)[6][6], double (&y)[6], double (&beta)[6]) {
  int perm[6] = {0, 1, 2, 3, 4, 5};
  double dmax = 0.0;
  for (int i = 0; i < 6; ++i) { dmax = fmax(dmax, A[i][i]); beta[i] = 0.0; }
  const double tol = 1e-12 * dmax;
  int r = 0;
  for (; r < 6; ++r) {
    int q = r;
    for (int i = r + 1; i < 6; ++i) if (A[i][i] > A[q][q]) q = i;
    if (!(A[q][q] > tol)) break;
    if (q != r) {  // symmetric swap of rows/columns r and q (the factored part included)
      for (int j = 0; j < 6; ++j) { const double t = A[r][j]; A[r][j] = A[q][j]; A[q][j] = t; }
      for (int j = 0; j < 6; ++j) { const double t = A[j][r]; A[j][r] = A[j][q]; A[j][q] = t; }
      { const double t = y[r]; y[r] = y[q]; y[q] = t; }
      { const int t = perm[r]; perm[r] = perm[q]; perm[q] = t; }
    }
    const double d = sqrt(A[r][r]);
    A[r][r] = d;
    for (int i = r + 1; i < 6; ++i) A[i][r] /= d;               // column r of L
    for (int i = r + 1; i < 6; ++i)
      for (int j = r + 1; j <= i; ++j) {
        A[i][j] -= A[i][r] * A[j][r];                             // Schur complement
        A[j][i] = A[i][j];
      }
  }
  double z[6];
  for (int i = 0; i < r; ++i) {
    double s = y[i];
    for (int j = 0; j < i; ++j) s -= A[i][j] * z[j];
    z[i] = s / A[i][i];
  }
  for (int i = r - 1; i >= 0; --i) {
    double s = z[i];
    for (int j = i + 1; j < r; ++j) s -= A[j][i] * z[j];
    z[i] = s / A[i][i];
  }
  for (int i = 0; i < r; ++i) beta[perm[i]] = z[i];
  return r;
}

// Applies the exercise rule of date m (regression coefficients already solved) to a path.
__device__ __forceinline__ void lsm_exercise(const DevOpt& o, const float* __restrict__ b32, int32_t m,
                                             float x, float v, float& h_c, int32_t& t) {
  const float S = asset(o, x);
  const float h = intrinsic(o, S);
  if (h > 0.0f) {
    float phi[6];
    lsm_basis(o, S, v, phi);
    float cont = 0.0f;
#pragma unroll
    for (int i = 0; i < 6; ++i) cont = __builtin_fmaf(phi[i], b32[i], cont);
    if (h > cont) { h_c = h; t = m; }
  }
}

constexpr int kLsmSums = 28;  // 21 Gram entries (upper triangle), 6 right-hand sides, count

// One date n of the backward induction (n = N-1 .. 1):
//   (a) exercise at date n + 1 with the coefficients the previous launch solved;
//   (b) in-the-money regression sums at date n of the cash flow discounted to t_n;
//   (c) the last block to finish sums the per-block partials in FP64 in block order and
//       solves for the coefficients of date n.
template <int BLOCK>
__global__ __launch_bounds__(BLOCK) void lsm_step_kernel(DevOpt o, int32_t n, const float* __restrict__ xs,
                                                         const float* __restrict__ vs,
                                                         float* __restrict__ hcash, int32_t* __restrict__ tau,
                                                         LsmState st) {
  __shared__ float s_red[kLsmSums * (BLOCK / kWave)];
  __shared__ int32_t s_last;
  const uint32_t p = blockIdx.x * BLOCK + threadIdx.x;
  const bool live = p < (uint32_t)o.paths;
  const size_t P = (size_t)o.paths;
  float h_c = 0.0f;
  int32_t t = 0;
  if (live) { h_c = hcash[p]; t = tau[p]; }
  const int32_t m = n + 1;
  if (m <= o.steps - 1) {
    const float* b32 = st.beta32 + (size_t)m * 8;
    if (b32[6] != 0.0f && live) {
      const int32_t t0 = t;
      lsm_exercise(o, b32, m, xs[(size_t)(m - 1) * P + p], vs[(size_t)(m - 1) * P + p], h_c, t);
      if (t != t0) { hcash[p] = h_c; tau[p] = t; }
    }
  }
  float acc[kLsmSums];
#pragma unroll
  for (int i = 0; i < kLsmSums; ++i) acc[i] = 0.0f;
  if (live) {
    const float S = asset(o, xs[(size_t)(n - 1) * P + p]);
    const float h = intrinsic(o, S);
    if (h > 0.0f) {
      float phi[6];
      lsm_basis(o, S, vs[(size_t)(n - 1) * P + p], phi);
      const float y = h_c * discount(o, t - n);
      int k = 0;
#pragma unroll
      for (int i = 0; i < 6; ++i)
#pragma unroll
        for (int j = i; j < 6; ++j) acc[k++] = phi[i] * phi[j];
#pragma unroll
      for (int i = 0; i < 6; ++i) acc[21 + i] = phi[i] * y;
      acc[27] = 1.0f;
    }
  }
  block_sum<BLOCK, kLsmSums, float>(acc, s_red);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < kLsmSums; ++i) st.gpart[(size_t)blockIdx.x * 32 + i] = acc[i];
    __threadfence();
    const uint32_t prev = atomicAdd(st.ticket, 1u);
    s_last = (prev == gridDim.x - 1);
  }
  __syncthreads();
  if (!s_last) return;
  __threadfence();
  // (c) fixed-order FP64 sum over blocks: thread (g, c) adds rows g, g + 8, ... of column c
  __shared__ double s_col[8 * 32];
  const int c = threadIdx.x & 31, g = threadIdx.x >> 5;
  if (g < 8 && c < kLsmSums) {
    double s = 0.0;
    for (uint32_t r = g; r < gridDim.x; r += 8) s += (double)st.gpart[(size_t)r * 32 + c];
    s_col[g * 32 + c] = s;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double tot[kLsmSums];
    for (int i = 0; i < kLsmSums; ++i) {
      double s = s_col[i];
      for (int gg = 1; gg < 8; ++gg) s += s_col[gg * 32 + i];
      tot[i] = s;
    }
    double A[6][6], yv[6], beta[6];
    int k = 0;
    for (int i = 0; i < 6; ++i)
      for (int j = i; j < 6; ++j) { A[i][j] = tot[k]; A[j][i] = tot[k]; ++k; }
    for (int i = 0; i < 6; ++i) yv[i] = tot[21 + i];
    float* b32 = st.beta32 + (size_t)n * 8;
    double* b64 = st.beta64 + (size_t)n * 6;
    if (tot[27] < 6.0) {
      for (int i = 0; i < 6; ++i) { b32[i] = 0.0f; b64[i] = 0.0; }
      b32[6] = 0.0f;
      atomicOr(st.flags, 1);
    } else {
      const int rank = solve_normal6(A, yv, beta);
      for (int i = 0; i < 6; ++i) { b32[i] = (float)beta[i]; b64[i] = beta[i]; }
      b32[6] = 1.0f;
      if (rank < 6) atomicOr(st.flags, 2);
    }
    *st.ticket = 0u;  // ready for the next date's launch
  }
}

// ---------------------------------------------------------------------------------------------
// The Gram matrices of all dates, before the backward induction.  The in-the-money set and the
// basis at date n depend only on the path states at n, so sum phi phi^T (and the count) of every
// date can be accumulated and factored ahead of time, in parallel across dates; the sequential
// induction then only reduces the 6 right-hand sides sum phi y, which depend on the cash flows.
// ---------------------------------------------------------------------------------------------
constexpr int kGramSums = LsmLayout<6>::kSums;  // the 15 moments of the 6-function basis
constexpr int kGramRow = kLsmGramRow;             // floats per (date, chunk) row
constexpr int kFacRec = kLsmFacRec;  // doubles per date: M = G^+ (36, row-major), [48] rank, [49] count, [50] valid,
                                     // [51] e^{r n dt}

// Index of the moment sum a^p c^q (p + q <= 4) in a row of the 6-function basis: by degree
// d = p + q, then by q (0: the count; 1, 2: a, c; 3..5: a^2, a c, c^2; 6..9: degree 3; 10..14:
// degree 4).  The basis (1, a, a^2, c, a c, c^2) is a^e c^f with these exponents, so the Gram
// entry (i, j) is the moment of (e_i + e_j, f_i + f_j).
__host__ __device__ constexpr int gram_moment(int p, int q) { return (p + q) * (p + q + 1) / 2 + q; }
constexpr int kBasisE[6] = {0, 1, 2, 0, 1, 0};
constexpr int kBasisF[6] = {0, 0, 0, 1, 1, 2};

// Block (date n = blockIdx.x + 1, chunk blockIdx.y): FP32 sums per lane over the chunk's paths
// p = chunk * (BLOCK * per_lane) + k * BLOCK + lane, FP32 block sums, one row per (date, chunk).
// With 6 functions the sums are the 15 moments (the 21 Gram entries hold only 15 distinct
// monomials: 3 products and 14 accumulations per path instead of 20); with 10 the Gram's upper
// triangle.
// lsm_gram_chunks makes per_lane <= 16, so every lane issues all its loads at once: 32-bit byte
// offsets from the date's uniform row base, unconditional and in bounds (slots past the chunk or
// the last path read the last path and are masked out of the sums).  The variance coordinate is
// formed outside the in-the-money branch: a load used only inside it is sunk into the branch by
// the compiler and waited for there, a full memory round trip per batch.
constexpr int kGramMaxPerLane = 16;

template <int BLOCK, int NB>
__global__ __launch_bounds__(BLOCK) void lsm_gram_kernel(DevOpt o, const float* __restrict__ xs,
                                                         const float* __restrict__ vs, int32_t per_lane,
                                                         float* __restrict__ gram) {
  constexpr int kGramSums = LsmLayout<NB>::kSums;
  constexpr int kGramRow = LsmLayout<NB>::kRow;
  __shared__ float s_red[kGramSums * (BLOCK / kWave)];
  const int n = blockIdx.x + 1;
  const size_t P = (size_t)o.paths;
  float acc[kGramSums];
#pragma unroll
  for (int i = 0; i < kGramSums; ++i) acc[i] = 0.0f;
  const uint32_t p0 = blockIdx.y * (uint32_t)(BLOCK * per_lane) + threadIdx.x;
  const uint32_t plast = (uint32_t)o.paths - 1;
  const SIMR_GLOBAL float* __restrict__ xr = as_global(xs) + (size_t)(n - 1) * P;
  const SIMR_GLOBAL float* __restrict__ vr = as_global(vs) + (size_t)(n - 1) * P;
  float xb[kGramMaxPerLane], vb[kGramMaxPerLane];
  bool ok[kGramMaxPerLane];
#pragma unroll
  for (int j = 0; j < kGramMaxPerLane; ++j) {
    const uint32_t p = p0 + (uint32_t)j * BLOCK;
    ok[j] = j < per_lane && p <= plast;
    const uint32_t boff = (p <= plast ? p : plast) * (uint32_t)sizeof(float);
    xb[j] = spill_at(xr, 0, boff);
    vb[j] = spill_at(vr, 0, boff);
  }
#pragma unroll
  for (int j = 0; j < kGramMaxPerLane; ++j) {
    float S = asset(o, xb[j]);
    float c = lsm_c(o, vb[j]);
    asm volatile("" : "+v"(S), "+v"(c));  // formed here, in path order, not inside the branch
    if (ok[j] && intrinsic(o, S) > 0.0f) {
      if constexpr (NB == 6) {
        const float a = lsm_a(o, S);
        const float a2 = a * a, ac = a * c, c2 = c * c;
        acc[gram_moment(0, 0)] += 1.0f;
        acc[gram_moment(1, 0)] += a;
        acc[gram_moment(0, 1)] += c;
        acc[gram_moment(2, 0)] += a2;
        acc[gram_moment(1, 1)] += ac;
        acc[gram_moment(0, 2)] += c2;
        acc[gram_moment(3, 0)] = __builtin_fmaf(a, a2, acc[gram_moment(3, 0)]);
        acc[gram_moment(2, 1)] = __builtin_fmaf(a, ac, acc[gram_moment(2, 1)]);
        acc[gram_moment(1, 2)] = __builtin_fmaf(a, c2, acc[gram_moment(1, 2)]);
        acc[gram_moment(0, 3)] = __builtin_fmaf(c, c2, acc[gram_moment(0, 3)]);
        acc[gram_moment(4, 0)] = __builtin_fmaf(a2, a2, acc[gram_moment(4, 0)]);
        acc[gram_moment(3, 1)] = __builtin_fmaf(a2, ac, acc[gram_moment(3, 1)]);
        acc[gram_moment(2, 2)] = __builtin_fmaf(a2, c2, acc[gram_moment(2, 2)]);
        acc[gram_moment(1, 3)] = __builtin_fmaf(ac, c2, acc[gram_moment(1, 3)]);
        acc[gram_moment(0, 4)] = __builtin_fmaf(c2, c2, acc[gram_moment(0, 4)]);
      } else {
        float phi[NB];
        lsm_basis_nb_ac<NB>(lsm_a(o, S), c, phi);
        // entry (0, 0) is phi_0^2 = 1 per path, the in-the-money count: summed once, below
        int q = 1;
#pragma unroll
        for (int a = 0; a < NB; ++a)
#pragma unroll
          for (int b = (a == 0 ? 1 : a); b < NB; ++b) { acc[q] = __builtin_fmaf(phi[a], phi[b], acc[q]); ++q; }
        acc[kGramSums - 1] += 1.0f;
      }
    }
  }
  if constexpr (NB != 6) acc[0] = acc[kGramSums - 1];
  block_sum<BLOCK, kGramSums, float>(acc, s_red);
  if (threadIdx.x == 0) {
    float* row = gram + ((size_t)n * gridDim.y + blockIdx.y) * kGramRow;
#pragma unroll
    for (int i = 0; i < kGramSums; ++i) row[i] = acc[i];
  }
}

__device__ __forceinline__ double readlane_d(double x, int l) {
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), l);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// One block per date n = blockIdx.x + 1.  The chunk rows are summed in FP64 in a fixed order:
// thread t adds rows t, t + 256, ... (each row read at once in 16-byte loads, so a date's rows
// arrive in one memory round trip instead of one per 8 chunks), each wave sums its lanes by a
// fixed butterfly, and lane e of wave 0 adds the four waves' partials of entry e in wave order.
// (One wave summing the rows in chunk order, 8 loads in flight, took 74 us per launch at 256
// chunks per date.)  Then wave 0 alone: the pivoted Cholesky factorisation P G P^T = L L^T in
// FP64 with lane 6 i + j holding entry (i, j).
// The pivot is the largest remaining Schur diagonal (lowest index on ties); once it is <= 1e-12
// times the largest original diagonal the remaining columns are dropped (rank < 6).  Dates with
// fewer than 6 in-the-money paths get no regression.  Record: the FP64 inverse on the kept
// columns, M = P^T (L L^T)^{-1} P (36), rank, count, valid.
constexpr int kFactorThreads = 256;

__global__ __launch_bounds__(kFactorThreads) void lsm_factor_kernel(int32_t chunks, double rdt,
                                                                    const float* __restrict__ gram,
                                                                    double* __restrict__ fac,
                                                                    int32_t* __restrict__ flags) {
  constexpr int W = kFactorThreads / kWave;
  static_assert(kGramRow % 4 == 0 && kGramSums <= kGramRow, "rows of whole 16-byte words");
  __shared__ double s_part[kGramSums * W];
  const int n = blockIdx.x + 1;
  const int lane = threadIdx.x & (kWave - 1);
  const int wid = threadIdx.x / kWave;
  double part[kGramSums];
#pragma unroll
  for (int e = 0; e < kGramSums; ++e) part[e] = 0.0;
  const float* rows = gram + (size_t)n * chunks * kGramRow;
  for (int c = threadIdx.x; c < chunks; c += kFactorThreads) {
    const float4* r4 = reinterpret_cast<const float4*>(rows + (size_t)c * kGramRow);
    float q[kGramRow];
#pragma unroll
    for (int k = 0; k < kGramRow / 4; ++k) {
      const float4 t = r4[k];
      q[4 * k] = t.x;
      q[4 * k + 1] = t.y;
      q[4 * k + 2] = t.z;
      q[4 * k + 3] = t.w;
    }
#pragma unroll
    for (int e = 0; e < kGramSums; ++e) part[e] += (double)q[e];
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1)  // each step on every entry before the next
#pragma unroll
    for (int e = 0; e < kGramSums; ++e) part[e] += __shfl_xor(part[e], off, kWave);
  if (lane == 0) {
#pragma unroll
    for (int e = 0; e < kGramSums; ++e) s_part[e * W + wid] = part[e];
  }
  __syncthreads();
  if (wid != 0) return;
  double sum = 0.0;
  if (lane < kGramSums) {
    sum = s_part[lane * W];
    for (int w = 1; w < W; ++w) sum += s_part[lane * W + w];
  }
  const double count = readlane_d(sum, gram_moment(0, 0));
  double* rec = fac + (size_t)n * kFacRec;
  if (count < 6.0) {
    if (lane < kFacRec) rec[lane] = 0.0;
    if (lane == 0) {
      rec[50] = 0.0;  // valid = 0: no exercise at this date
      atomicOr(flags, 1);
    }
    return;
  }
  const int i = lane / 6, j = lane - 6 * (lane / 6);
  const bool in = lane < 36;
  const int src = in ? gram_moment(kBasisE[i] + kBasisE[j], kBasisF[i] + kBasisF[j]) : 0;
  double a = __shfl(sum, src, kWave);
  if (!in) a = 0.0;
  int perm = lane;
  double dmax = 0.0;
#pragma unroll
  for (int c = 0; c < 6; ++c) dmax = fmax(dmax, readlane_d(a, 7 * c));
  const double tol = 1e-12 * dmax;
  int rank = 6;
#pragma unroll
  for (int r = 0; r < 6; ++r) {
    int q = r;
    double best = readlane_d(a, 7 * r);
#pragma unroll
    for (int c = r + 1; c < 6; ++c) {
      const double d = readlane_d(a, 7 * c);
      if (d > best) { best = d; q = c; }
    }
    if (!(best > tol)) { rank = r; break; }
    if (q != r) {
      const int pi = (i == r) ? q : (i == q ? r : i);
      const int pj = (j == r) ? q : (j == q ? r : j);
      a = __shfl(a, in ? pi * 6 + pj : lane, kWave);
      const int pl = (lane == r) ? q : (lane == q ? r : lane);
      perm = __shfl(perm, pl, kWave);
    }
    const double d = sqrt(readlane_d(a, 7 * r));
    const double id = 1.0 / d;
    if (in && j == r && i > r) a *= id;
    if (lane == 7 * r) a = d;
    const double lir = __shfl(a, in ? i * 6 + r : lane, kWave);
    const double ljr = __shfl(a, in ? j * 6 + r : lane, kWave);
    if (in && i > r && j > r) a -= lir * ljr;
  }
  // M = P^T (L L^T)^{-1} P on the kept columns (zero rows/columns for dropped ones), so that
  // the induction's solve is beta = M y.  Lane 0 inverts the triangular factor: W = L^{-1},
  // (L L^T)^{-1} = W^T W.
  double Lr[6][6];
#pragma unroll
  for (int r = 0; r < 6; ++r)
#pragma unroll
    for (int c = 0; c < 6; ++c) Lr[r][c] = (c <= r) ? readlane_d(a, r * 6 + c) : 0.0;
  int pr[6];
#pragma unroll
  for (int c = 0; c < 6; ++c) pr[c] = __builtin_amdgcn_readlane(perm, c);
  if (lane == 0) {
    double W[6][6];
#pragma unroll
    for (int r = 0; r < 6; ++r)
#pragma unroll
      for (int c = 0; c < 6; ++c) W[r][c] = 0.0;
#pragma unroll
    for (int c = 0; c < 6; ++c) {  // column c of W: L W[:, c] = e_c
      if (c < rank) {
        W[c][c] = 1.0 / Lr[c][c];
#pragma unroll
        for (int r = c + 1; r < 6; ++r) {
          if (r < rank) {
            double t = 0.0;
#pragma unroll
            for (int q = c; q < r; ++q) t += Lr[r][q] * W[q][c];
            W[r][c] = -t / Lr[r][r];
          }
        }
      }
    }
    double M[6][6];
#pragma unroll
    for (int i = 0; i < 6; ++i)
#pragma unroll
      for (int j = 0; j < 6; ++j) {
        double t = 0.0;
#pragma unroll
        for (int q = 0; q < 6; ++q) t += W[q][i] * W[q][j];
        M[i][j] = t;
      }
    for (int i = 0; i < 36; ++i) rec[i] = 0.0;
#pragma unroll
    for (int i = 0; i < 6; ++i)
#pragma unroll
      for (int j = 0; j < 6; ++j)
        if (i < rank && j < rank) rec[pr[i] * 6 + pr[j]] = M[i][j];
    rec[48] = (double)rank;
    rec[49] = count;
    rec[50] = 1.0;
    rec[51] = exp(rdt * (double)n);
    if (rank < 6) atomicOr(flags, 2);
  }
}

// The same record for a basis of NB functions (NB = 10): the lanes sum the chunk rows as above,
// then factor and invert in FP64 with the matrix in LDS, one entry per lane at each step (the
// pivot choice, swaps, column scaling and Schur update of every step in parallel, one column of
// L^{-1} per lane, the entries of M two per lane); each entry takes the same operations in the
// same order as a serial elimination, with the same pivot and drop rule as the 6-function one.
template <int NB>
__global__ __launch_bounds__(64) void lsm_factor_serial_kernel(int32_t chunks, double rdt,
                                                               const float* __restrict__ gram,
                                                               double* __restrict__ fac, int32_t* __restrict__ flags) {
  using LL = LsmLayout<NB>;
  static_assert(NB * NB <= 2 * kWave && LL::kSums <= kWave, "one wave, at most two entries per lane");
  __shared__ double s_sum[64];
  __shared__ double A[NB][NB + 1];
  __shared__ double Wm[NB][NB + 1];
  __shared__ int perm[NB];
  const int n = blockIdx.x + 1;
  const int lane = threadIdx.x;
  double sum = 0.0;
  if (lane < LL::kSums) {
    const float* rows = gram + (size_t)n * chunks * LL::kRow + lane;
    for (int c0 = 0; c0 < chunks; c0 += 8) {  // 8 loads in flight, summed in chunk order
      float v[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) v[j] = c0 + j < chunks ? rows[(size_t)(c0 + j) * LL::kRow] : 0.0f;
#pragma unroll
      for (int j = 0; j < 8; ++j)
        if (c0 + j < chunks) sum += (double)v[j];
    }
  }
  s_sum[lane] = sum;
  double* rec = fac + (size_t)n * LL::kRec;
  for (int i = lane; i < LL::kRec; i += kWave) rec[i] = 0.0;
  __syncthreads();
  const double count = s_sum[LL::kSums - 1];
  if (count < (double)NB) {  // valid stays 0: no exercise at this date
    if (lane == 0) atomicOr(flags, 1);
    return;
  }
  if (lane < LL::kSums - 1) {  // upper-triangle entry q = lane -> (a, b), row order
    int a = 0, rem = lane;
    while (rem >= NB - a) {
      rem -= NB - a;
      ++a;
    }
    A[a][a + rem] = s_sum[lane];
    A[a + rem][a] = s_sum[lane];
  }
  if (lane < NB) perm[lane] = lane;
  __syncthreads();
  double dmax = 0.0;
  for (int i = 0; i < NB; ++i) dmax = fmax(dmax, A[i][i]);
  const double tol = 1e-12 * dmax;
  int rank = 0;
  for (; rank < NB; ++rank) {  // P A P^T = L L^T, L kept in the lower triangle of A
    const int r = rank;
    int q = r;
    for (int i = r + 1; i < NB; ++i)
      if (A[i][i] > A[q][q]) q = i;
    if (!(A[q][q] > tol)) break;
    if (q != r) {
      if (lane < NB) {
        const double t = A[r][lane];
        A[r][lane] = A[q][lane];
        A[q][lane] = t;
      }
      __syncthreads();
      if (lane < NB) {
        const double t = A[lane][r];
        A[lane][r] = A[lane][q];
        A[lane][q] = t;
      }
      if (lane == 0) {
        const int t = perm[r];
        perm[r] = perm[q];
        perm[q] = t;
      }
      __syncthreads();
    }
    const double dd = sqrt(A[r][r]);
    __syncthreads();
    if (lane == r) A[r][r] = dd;
    if (lane > r && lane < NB) A[lane][r] /= dd;
    __syncthreads();
    const int m = NB - r - 1;  // Schur complement entries (i, j), r < j <= i < NB
    for (int e = lane; e < m * (m + 1) / 2; e += kWave) {
      int i = 0, rem = e;
      while (rem > i) {
        rem -= i + 1;
        ++i;
      }
      const int ii = r + 1 + i, jj = r + 1 + rem;
      const double v = A[ii][jj] - A[ii][r] * A[jj][r];
      A[ii][jj] = v;
      A[jj][ii] = v;
    }
    __syncthreads();
  }
  // W = L^{-1} on the kept columns (lane c: column c); M = P^T W^T W P
  if (lane < NB) {
    for (int r = 0; r < NB; ++r) Wm[r][lane] = 0.0;
    const int c = lane;
    if (c < rank) {
      Wm[c][c] = 1.0 / A[c][c];
      for (int r = c + 1; r < rank; ++r) {
        double t = 0.0;
        for (int qq = c; qq < r; ++qq) t += A[r][qq] * Wm[qq][c];
        Wm[r][c] = -t / A[r][r];
      }
    }
  }
  __syncthreads();
  for (int e = lane; e < rank * rank; e += kWave) {
    const int i = e / rank, j = e % rank;
    double t = 0.0;
    for (int qq = 0; qq < rank; ++qq) t += Wm[qq][i] * Wm[qq][j];
    rec[perm[i] * NB + perm[j]] = t;
  }
  if (lane == 0) {
    rec[LL::kRank] = (double)rank;
    rec[LL::kRank + 1] = count;
    rec[LL::kRank + 2] = 1.0;
    rec[LL::kRank + 3] = exp(rdt * (double)n);
    if (rank < NB) atomicOr(flags, 2);
  }
}

// Exchange of the per-block right-hand-side sums for date k (k = 1, 2, ...) without counters or
// fences: block b publishes each of its 6 FP32 sums as one 64-bit word (k << 32 | float bits) at
// slot [k & 1][b][c] with a relaxed agent-scope atomic store, and readers poll those words with
// relaxed agent-scope atomic loads until every one carries tag k.  Tag and value travel in one
// single-copy-atomic word, so a word that shows tag k holds date k's value; the two parity
// buffers keep a block that is a date ahead from overwriting a word still being read (to write
// date k + 2 it must have read everyone's date k + 1, written after they finished date k).  The
// words are zeroed before the launch.  The wait is bounded: on a timeout the status word is set
// and later waits give up at once.
constexpr uint32_t kSpinLimit = 1u << 22;  // passes (a few seconds of polling) before a wait gives up

// Called by a whole wave with the row uniform across it: lane c < NB stores word c, so the row
// leaves as one write instruction (NB stores issued one after another by a single lane took 6%
// longer per C2 pricing pass: the readers wait for the last word of every row).
template <int NB>
__device__ __forceinline__ void xchg_publish(SIMR_GLOBAL unsigned long long* slot, const float (&v)[NB], uint32_t k) {
  const int lane = threadIdx.x & (kWave - 1);
  float mine = v[0];
#pragma unroll
  for (int c = 1; c < NB; ++c) mine = lane == c ? v[c] : mine;
  if (lane < NB) {
    const unsigned long long w = ((unsigned long long)k << 32) | (unsigned long long)__float_as_uint(mine);
    __hip_atomic_store(slot + lane, w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// Another lane's value of a double (DPP control CTRL within each 16-lane row), both halves moved.
template <int CTRL>
__device__ __forceinline__ double dpp_term_d(double x) {
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffll), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Read by one wave of the pollers: with XW words per block row and GR = 64 / XW groups, lane
// (c, g) = (lane / GR, lane % GR) polls column c < NB of the rows row0 + g + GR m, m < 8 (all 8
// loads of a lane in flight at once, so a pass over the wave's 8 GR rows is one memory round
// trip), and sums them in FP64 in increasing m; pairwise sums over g ^ 1, g ^ 2 (and g ^ 4) by
// DPP inside the lane's row then leave every lane of column c holding the sum over the wave's
// rows (lanes c GR .. c GR + GR - 1).  A task of G blocks takes ceil(G / (8 GR)) pollers per
// block, each on its own 8 GR rows: one wave for up to 64 blocks (32 with 16 words per row), and
// the passes of the pollers of a larger task run side by side instead of one after another.
// The order is fixed, so every block obtains the same bits.  The exchange is bound by the time
// from the last row landing to the poller seeing it: a pass loads the status word together with
// its rows and the next pass follows without a pause.  Redundant pollers (several waves racing
// over the same rows), or a pause between passes, measured slower: the extra loads contend
// with the rows being published.
template <int XW, int NB>
__device__ __forceinline__ double xchg_gather(const SIMR_GLOBAL unsigned long long* buf, uint32_t G, uint32_t row0, uint32_t k,
                                              int32_t* status) {
  constexpr uint32_t GR = kWave / XW;
  static_assert(GR == 4 || GR == 8, "the groups of a column lie in one half-row");
  const int lane = threadIdx.x & (kWave - 1);
  const uint32_t g = (uint32_t)lane % GR, c = (uint32_t)lane / GR;
  double acc = 0.0;
  const SIMR_GLOBAL char* base = (const SIMR_GLOBAL char*)buf;
  // the 32-bit byte offsets of the lane's rows from the uniform base (rows past G read row
  // G - 1, in bounds; their values are not used)
  uint32_t off[8];
#pragma unroll
  for (int m = 0; m < 8; ++m) {
    const uint32_t r = row0 + g + GR * m;
    off[m] = ((r < G ? r : G - 1) * XW + c) * (uint32_t)sizeof(unsigned long long);
  }
  if (c < NB) {
    uint32_t spins = 0;
    for (;;) {  // a pass reads the wave's rows; it is repeated until all carry tag k
      const int32_t failed = __hip_atomic_load(status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      bool ready = true;
      double s = 0.0;
      unsigned long long w[8];
#pragma unroll
      for (int m = 0; m < 8; ++m) {
        // The empty statement makes the offset a value of this pass, so the address is formed
        // here as scalar base + 32-bit offset.  Otherwise the compiler hoists eight 64-bit
        // addresses out of the loop, 16 registers that 16 waves per CU cannot hold, and their
        // spill reloads make the poll wait for every load in flight.
        uint32_t o = off[m];
        asm volatile("" : "+v"(o));
        w[m] = __hip_atomic_load((const SIMR_GLOBAL unsigned long long*)(base + o), __ATOMIC_RELAXED,
                                 __HIP_MEMORY_SCOPE_AGENT);
      }
#pragma unroll
      for (int m = 0; m < 8; ++m) {
        const bool in = row0 + g + GR * m < G;
        ready &= !in || (uint32_t)(w[m] >> 32) == k;
        s += in ? (double)__uint_as_float((uint32_t)w[m]) : 0.0;
      }
      if (ready) {
        acc = s;
        break;
      }
      if (failed != 0) break;
      if (++spins > kSpinLimit) {
        atomicOr(status, 1);
        break;
      }
    }
  }
  acc += dpp_term_d<0xB1>(acc);                          // quad_perm [1,0,3,2]: g ^ 1
  acc += dpp_term_d<0x4E>(acc);                          // quad_perm [2,3,0,1]: g ^ 2
  if constexpr (GR == 8) acc += dpp_term_d<0x141>(acc);  // row_half_mirror: the other quad
  return acc;
}

// Sum over each 16-lane row of the wave by DPP (every lane of the row holds its row's sum).
__device__ __forceinline__ float row_sum16(float x) {
  x += dpp_term<0xB1, 0xF>(x);   // quad_perm [1,0,3,2]
  x += dpp_term<0x4E, 0xF>(x);   // quad_perm [2,3,0,1]
  x += dpp_term<0x141, 0xF>(x);  // row_half_mirror
  x += dpp_term<0x140, 0xF>(x);  // row_mirror
  return x;
}

// s_waitcnt vmcnt(0) in the gfx9 encoding (vmcnt 0; expcnt 7 and lgkmcnt 15, which do not wait).
constexpr int kWaitVmcnt0 = 0x0F70;

// Paths per block fix the induction's bits, the block size does not: a block of BLOCK threads
// sums its paths as kLsmVBlock virtual lanes (virtual lane s BLOCK + lane holds paths j of the
// lane with j % S == s, S = kLsmVBlock / BLOCK, in increasing j), each 16 virtual lanes a row,
// so 256 threads with 16 paths per lane give the bits of 1024 threads with 4: the same sums in
// the same order.  The smaller blocks fit twice as many per CU, so two options of 2^20 paths
// can share one launch.
constexpr int kLsmVBlock = 1024;

// The backward induction in one cooperative launch (all blocks co-resident).  The launch carries
// one or more options (tasks), each on its own consecutive blocks (at most 256), so the
// inductions of several options run side by side and hide each other's exchange latency.
// Every lane owns PPL paths of its task (path = b * BLOCK * PPL + j * BLOCK + lane, b the block
// within the task) and keeps their exercise index tau and cash flow, as its value at t_0, in
// registers for the whole induction, reading each date's spilled (x_n, v_n) once, two dates
// ahead.  A date n: FP32 right-hand-side sums of phi times the t_0 values per lane and per block
// -> tagged exchange of the task's block rows (while it is in flight the lanes already evaluate
// the basis coordinates of date n - 1) -> every block of the task sums all rows in the same
// fixed order in FP64 -> beta from the precomputed factor of the date, times e^{r n dt} (the
// right-hand side discounted to date n) -> exercise update.
//   Wait counts shape this kernel.  A wave's vector-memory counter retires its loads (and
// stores) in the order they were issued, so consuming one load waits for every access issued
// before it; the code below is arranged so that no wave waits, before its poll or at a barrier,
// for the spill rows it requested for a later date.
template <int BLOCK, int PPL, int NB>
__global__ __launch_bounds__(BLOCK) void lsm_persistent_kernel(
    const LsmTask* __restrict__ tasks, int32_t ntasks,
                                                               int32_t* __restrict__ status) {
  using LL = LsmLayout<NB>;
  constexpr int W = BLOCK / kWave;
  constexpr int S = kLsmVBlock / BLOCK;  // virtual lanes per lane
  constexpr int R = kLsmVBlock / 16;     // 16-lane rows of the virtual block
  constexpr uint32_t kRowsPerPoller = 8 * (kWave / LL::kXW);
  static_assert(kLsmVBlock % BLOCK == 0 && PPL % S == 0, "whole virtual lanes per lane");
  static_assert(R == kWave, "one wave folds the row partials");
  static_assert(W * kRowsPerPoller >= 256, "enough pollers for the largest task (256 blocks)");
  __shared__ float s_red[NB * R];
  __shared__ double s_bq[W * NB];  // each poller's share of beta: e^{r n dt} M times its rows' sums
  __shared__ double s_valid;       // nonzero: the date has a regression (wave 0, with its share)
  const int lane = threadIdx.x & (kWave - 1);
  // wave-uniform (the compiler does not infer it): the pollers' branch is a scalar branch, not
  // a masked one whose wait counts include the loads of the other branch
  const int wid = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / kWave));
  int32_t t = 0, hi = ntasks - 1;  // the last task whose first block is <= blockIdx.x
  while (t < hi) {
    const int32_t mid = (t + hi + 1) >> 1;
    if (tasks[mid].block0 <= (int32_t)blockIdx.x) t = mid; else hi = mid - 1;
  }
  const LsmTask& T = tasks[t];
  const DevOpt o = T.o;
  const SIMR_GLOBAL float* __restrict__ xs = as_global(T.xs);
  const SIMR_GLOBAL float* __restrict__ vs = as_global(T.vs);
  const SIMR_GLOBAL double* __restrict__ fac = as_global(T.fac);
  const uint32_t G = (uint32_t)T.nblocks;
  const uint32_t blk = blockIdx.x - (uint32_t)T.block0;
  const uint32_t npoll = (G + kRowsPerPoller - 1) / kRowsPerPoller;  // waves 0 .. npoll - 1 poll
  const int N = o.steps;
  const size_t P = (size_t)o.paths;
  // per path: the exercise index tau and w = e^{-r tau dt} h(S_tau), the cash flow's value at
  // t_0 (so the discounting of every date is one factor e^{r n dt} on the block sums).  Path j
  // of the lane is p_0 + j BLOCK, read from a date's spill row at the 32-bit byte offset 4 p_j
  // (paths <= 2^30) from the row's uniform base: one offset register per path instead of a
  // 64-bit address per path and array.  A lane past the last path reads the last path (in
  // bounds, unused) and holds S = K, so h(S) = 0 and it never enters a sum or the exercise.
  const uint32_t p0 = blk * (BLOCK * PPL) + threadIdx.x;
  bool live[PPL];
  uint32_t boff[PPL];
  float w[PPL];
  int32_t tu[PPL];
  const float dN = discount(o, N);
#pragma unroll
  for (int j = 0; j < PPL; ++j) {
    live[j] = p0 + j * BLOCK < (uint32_t)o.paths;
    boff[j] = (live[j] ? p0 + j * BLOCK : (uint32_t)o.paths - 1) * (uint32_t)sizeof(float);
    w[j] = live[j] ? intrinsic(o, asset(o, spill_at(xs, (size_t)(N - 1) * P, boff[j]))) * dN : 0.0f;
    tu[j] = N;
  }
  // date n state: h = h(S) and the basis coordinates a = (S - K) / K, c = (max(v, 0) - theta) /
  // theta, evaluated once per date in the exchange window of the date before and used by both
  // the sums and the exercise (the same operations as forming them from S and v where they are
  // used, so the same values); raw (x, v) of date n - 1 already requested
  float hn[PPL], an[PPL], cn[PPL], xq[PPL], vq[PPL];
  // Every request is unconditional and in bounds (rows before the first date read row 0, their
  // values unused): a request under a condition leaves the old and the new value meeting at the
  // join, where the compiler copies the new one and so waits for it two dates early.
  {
    const size_t r2 = (size_t)(N >= 2 ? N - 2 : 0) * P, r3 = (size_t)(N >= 3 ? N - 3 : 0) * P;
#pragma unroll
    for (int j = 0; j < PPL; ++j) {
      const float x = spill_at(xs, r2, boff[j]);
      cn[j] = lsm_c(o, spill_at(vs, r2, boff[j]));
      const float S = live[j] ? asset(o, x) : o.K;
      hn[j] = intrinsic(o, S);
      an[j] = lsm_a(o, S);
      xq[j] = spill_at(xs, r3, boff[j]);
      vq[j] = spill_at(vs, r3, boff[j]);
    }
  }
  for (int32_t n = N - 1; n >= 1; --n) {
    // (b) right-hand-side sums at date n over t_0 values, per virtual lane; 16-lane row sums ->
    // LDS (virtual row s W 4 + wid 4 + lane / 16); wave 0 folds the rows and publishes them
#pragma unroll
    for (int s = 0; s < S; ++s) {
      float acc[NB];
#pragma unroll
      for (int a = 0; a < NB; ++a) acc[a] = 0.0f;
#pragma unroll
      for (int j = s; j < PPL; j += S) {
        if (hn[j] > 0.0f) {
          float phi[NB];
          lsm_basis_nb_ac<NB>(an[j], cn[j], phi);
#pragma unroll
          for (int a = 0; a < NB; ++a) acc[a] = __builtin_fmaf(phi[a], w[j], acc[a]);
        }
      }
#pragma unroll
      for (int a = 0; a < NB; ++a) acc[a] = row_sum16(acc[a]);
      if ((lane & 15) == 0) {
#pragma unroll
        for (int a = 0; a < NB; ++a) s_red[a * R + s * 4 * W + wid * 4 + (lane >> 4)] = acc[a];
      }
    }
    __syncthreads();
    const uint32_t k = (uint32_t)(N - n);
    SIMR_GLOBAL unsigned long long* buf = as_global(T.xchg) + (size_t)(k & 1) * G * LL::kXW;
    // The solve of date n does not depend on the induction.  The pollers read its record once
    // the block's sums are folded (lane i < NB: row i of M; e^{r n dt}; the valid flag, which
    // wave 0 passes on through LDS).  Only the pollers wait for these loads: a vector load in
    // every wave would make each wait for its requests of date n - 2 as well, since the
    // vector-memory counter retires loads in the order they were issued.
    double mrow[NB], grow = 0.0, mvalid = 0.0;
    if ((uint32_t)wid < npoll) {
#pragma unroll
      for (int c = 0; c < NB; ++c) mrow[c] = lane < NB ? fac[(size_t)n * LL::kRec + lane * NB + c] : 0.0;
      grow = fac[(size_t)n * LL::kRec + LL::kRank + 3];
      mvalid = fac[(size_t)n * LL::kRec + LL::kRank + 2];
    }
    if (wid == 0) {
      float row[NB];
#pragma unroll
      for (int a = 0; a < NB; ++a) row[a] = s_red[a * R + lane];
      wave_sum_n<NB>(row);  // the NB folds interleaved
      xchg_publish<NB>(buf + (size_t)blk * LL::kXW, row, k);
    }
    // while the rows travel: evaluate h, a and c of date n - 1, then request date n - 2.  The
    // empty statement takes the new coordinates and hands on the offset, so the requests go out
    // only once the old (x, v) are consumed and can land in the same registers; otherwise the
    // compiler issues them first and copies them into place at the end of the date, a copy
    // that waits for them.  (Issued after the second barrier instead, the requests measured
    // slower: 2.3 -> 2.7 us per date at 131,072 paths, 3.9 -> 4.6 us at 2^20.)
    float h1[PPL], a1[PPL], c1[PPL];
    const size_t r3 = (size_t)(n >= 3 ? n - 3 : 0) * P;
#pragma unroll
    for (int j = 0; j < PPL; ++j) {
      const float S = live[j] ? asset(o, xq[j]) : o.K;
      h1[j] = intrinsic(o, S);
      a1[j] = lsm_a(o, S);
      c1[j] = lsm_c(o, vq[j]);
      uint32_t b = boff[j];
      asm volatile("" : "+v"(b) : "v"(h1[j]), "v"(a1[j]), "v"(c1[j]));
      xq[j] = spill_at(xs, r3, b);
      vq[j] = spill_at(vs, r3, b);
    }
    // (c) the pollers: poller q sums the rows of its blocks in a fixed order in FP64 (y_q, lane
    // c GR holding column c) and leaves its share beta_q,i = e^{r n dt} sum_c M_ic y_q,c (lane i)
    // in LDS; then lane i of every wave adds the shares in poller order, beta_i = sum_q
    // beta_q,i.  With one poller (up to 64 blocks) that is the solve beta = e^{r n dt} M y
    // itself.  The same operations in every wave and block give every block the same bits.
    //   With several pollers per block (more than 64 blocks) each poller first waits for its
    // own requests of date n - 2.  Polling at once, 4 pollers in each of 256 blocks re-read all
    // 256 rows flat out while the date's 8 MB of spill rows stream in: at 2^20 paths a date
    // took 4.9 us so and 4.2 us with the wait (before the coordinates were held across dates).
    if ((uint32_t)wid < npoll) {
      if (npoll > 1) __builtin_amdgcn_s_waitcnt(kWaitVmcnt0);
      const double y = xchg_gather<LL::kXW, NB>(buf, G, (uint32_t)wid * kRowsPerPoller, k, status);
      double bq = 0.0;
#pragma unroll
      for (int c = 0; c < NB; ++c) bq = __builtin_fma(mrow[c], readlane_d(y, c * (kWave / LL::kXW)), bq);
      bq *= grow;  // the sums are of t_0 values: discount to date n
      if (lane < NB) s_bq[wid * NB + lane] = bq;
      if (wid == 0 && lane == 0) s_valid = mvalid;  // compared after the barrier
    }
    __syncthreads();
    const bool valid = s_valid != 0.0;
    // (a) exercise at date n
    if (valid) {
      // lane i < NB forms beta_i in FP64 and rounds it once; the wave then reads the NB
      // coefficients from those lanes as scalars.  (Every lane forming all NB sums, in all 16
      // waves, had made this the longest phase of a date: 1.4 of 5.4 us at 2^20 paths.)
      double beta = 0.0;
      if (lane < NB) {
        beta = s_bq[lane];
        for (uint32_t q = 1; q < npoll; ++q) beta += s_bq[q * NB + lane];
        if (wid == 0 && blk == 0 && T.beta64) as_global(T.beta64)[(size_t)n * NB + lane] = beta;
      }
      const float bl = (float)beta;
      float b[NB];
#pragma unroll
      for (int i = 0; i < NB; ++i) b[i] = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(bl), i));
      const float dn = discount(o, n);
#pragma unroll
      for (int j = 0; j < PPL; ++j) {
        const float h = hn[j];
        if (h > 0.0f) {
          float phi[NB];
          lsm_basis_nb_ac<NB>(an[j], cn[j], phi);
          float cont = 0.0f;
#pragma unroll
          for (int i = 0; i < NB; ++i) cont = __builtin_fmaf(phi[i], b[i], cont);
          if (h > cont) { w[j] = h * dn; tu[j] = n; }
        }
      }
    } else if (wid == 0 && lane < NB && blk == 0 && T.beta64) {
      as_global(T.beta64)[(size_t)n * NB + lane] = 0.0;
    }
#pragma unroll
    for (int j = 0; j < PPL; ++j) { hn[j] = h1[j]; an[j] = a1[j]; cn[j] = c1[j]; }
  }
  // discounted cash flows: Kahan in FP32 per virtual lane, FP64 across the block (the wave sums
  // of the virtual waves s W + wid, then their sum in virtual wave order)
  constexpr int VW = kLsmVBlock / kWave;
  __shared__ double s_red2[2 * VW];
#pragma unroll
  for (int s = 0; s < S; ++s) {
    Kahan k1, k2;
#pragma unroll
    for (int j = s; j < PPL; j += S) {
      if (live[j]) {
        const float X = w[j];  // h(S_tau) e^{-r tau dt}
        k1.add(X);
        k2.add(X * X);
        as_global(T.tau)[p0 + j * BLOCK] = tu[j];
      }
    }
    const double v1 = wave_sum(k1.value()), v2 = wave_sum(k2.value());
    if (lane == 0) {
      s_red2[s * W + wid] = v1;
      s_red2[VW + s * W + wid] = v2;
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double v1 = s_red2[0], v2 = s_red2[VW];
    for (int q = 1; q < VW; ++q) {
      v1 += s_red2[q];
      v2 += s_red2[VW + q];
    }
    as_global(T.partials)[2 * (size_t)blk] = v1;
    as_global(T.partials)[2 * (size_t)blk + 1] = v2;
  }
}

// The same induction with one launch per date, for a task whose paths cannot all be co-resident
// (it takes the factor records of the Gram pre-pass, as the cooperative kernel does).  One path
// per lane keeps w, the cash flow valued at t_0, and its exercise index in memory.  Date n's
// launch (n = N - 1, ..., 1): at n = N - 1 it sets w = e^{-r T} h(S_N) and tau = N; otherwise it
// applies the exercise at date n + 1 with that date's beta, written by the previous launch.  Then
// it sums phi_n w over the in-the-money paths of date n into one FP32 row per block; the last
// block to finish (a ticket) sums the rows in FP64 in block order and writes
// beta_n = e^{r n dt} M_n y, or marks the date without a regression.  beta32: LsmLayout<NB>::kXW
// floats per date (beta, then the valid flag at NB); gpart: kXW floats per block.
template <int NB>
__device__ __forceinline__ void lsm_date_exercise(const DevOpt& o, int32_t m, float x, float v,
                                                  const float* __restrict__ b, float& w, int32_t& tau) {
  const float S = asset(o, x);
  const float h = intrinsic(o, S);
  if (b[NB] != 0.0f && h > 0.0f) {
    float phi[NB];
    lsm_basis_nb<NB>(o, S, v, phi);
    float cont = 0.0f;
#pragma unroll
    for (int i = 0; i < NB; ++i) cont = __builtin_fmaf(phi[i], b[i], cont);
    if (h > cont) {
      w = h * discount(o, m);
      tau = m;
    }
  }
}

template <int BLOCK, int NB>
__global__ __launch_bounds__(BLOCK) void lsm_date_kernel(DevOpt o, int32_t n, const float* __restrict__ xs,
                                                         const float* __restrict__ vs, const double* __restrict__ fac,
                                                         float* __restrict__ wcash, int32_t* __restrict__ tau,
                                                         float* __restrict__ gpart, float* __restrict__ beta32,
                                                         double* __restrict__ beta64, uint32_t* __restrict__ ticket) {
  using LL = LsmLayout<NB>;
  constexpr int XW = LL::kXW;
  constexpr int GROUPS = BLOCK / XW;
  static_assert(NB <= XW && BLOCK % XW == 0, "layout");
  __shared__ float s_red[NB * (BLOCK / kWave)];
  __shared__ double s_col[BLOCK];
  __shared__ int32_t s_last;
  const uint32_t p = blockIdx.x * BLOCK + threadIdx.x;
  const bool live = p < (uint32_t)o.paths;
  const size_t P = (size_t)o.paths;
  const int N = o.steps;
  float w = 0.0f;
  int32_t t = N;
  if (live) {
    if (n == N - 1) {
      w = intrinsic(o, asset(o, xs[(size_t)(N - 1) * P + p])) * discount(o, N);
    } else {
      w = wcash[p];
      t = tau[p];
      const int32_t m = n + 1;
      lsm_date_exercise<NB>(o, m, xs[(size_t)(m - 1) * P + p], vs[(size_t)(m - 1) * P + p],
                            beta32 + (size_t)m * XW, w, t);
    }
    wcash[p] = w;
    tau[p] = t;
  }
  float acc[NB];
#pragma unroll
  for (int a = 0; a < NB; ++a) acc[a] = 0.0f;
  if (live) {
    const float S = asset(o, xs[(size_t)(n - 1) * P + p]);
    if (intrinsic(o, S) > 0.0f) {
      float phi[NB];
      lsm_basis_nb<NB>(o, S, vs[(size_t)(n - 1) * P + p], phi);
#pragma unroll
      for (int a = 0; a < NB; ++a) acc[a] = phi[a] * w;
    }
  }
  block_sum<BLOCK, NB, float>(acc, s_red);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int a = 0; a < NB; ++a) gpart[(size_t)blockIdx.x * XW + a] = acc[a];
    __threadfence();
    const uint32_t prev = atomicAdd(ticket, 1u);
    s_last = (prev == gridDim.x - 1);
  }
  __syncthreads();
  if (!s_last) return;
  __threadfence();
  // fixed-order FP64 sum over the block rows: thread (g, c) adds rows g, g + GROUPS, ... of
  // column c, then thread c adds the GROUPS partials in order
  const int c = threadIdx.x % XW, g = threadIdx.x / XW;
  double sum = 0.0;
  if (c < NB)
    for (uint32_t r = g; r < gridDim.x; r += GROUPS) sum += (double)gpart[(size_t)r * XW + c];
  s_col[threadIdx.x] = sum;
  __syncthreads();
  if (threadIdx.x < XW) {
    double y = 0.0;
    for (int gg = 0; gg < GROUPS; ++gg) y += s_col[gg * XW + threadIdx.x];
    s_col[threadIdx.x] = y;
  }
  __syncthreads();
  if (threadIdx.x < NB) {
    const double* rec = fac + (size_t)n * LL::kRec;
    const bool valid = rec[LL::kRank + 2] != 0.0;
    double beta = 0.0;
#pragma unroll
    for (int j = 0; j < NB; ++j) beta = __builtin_fma(rec[threadIdx.x * NB + j], s_col[j], beta);
    beta *= rec[LL::kRank + 3];  // the sums are of t_0 values: discount to date n
    beta32[(size_t)n * XW + threadIdx.x] = valid ? (float)beta : 0.0f;
    if (beta64) beta64[(size_t)n * NB + threadIdx.x] = valid ? beta : 0.0;
    if (threadIdx.x == 0) {
      beta32[(size_t)n * XW + NB] = valid ? 1.0f : 0.0f;
      *ticket = 0u;  // ready for the next date's launch
    }
  }
}

// The end of the per-date induction: the exercise at date 1 (or, with N = 1, the maturity cash
// flow), the exercise indices, and per block the FP64 sums of the t_0 cash flows and their
// squares (Kahan FP32 per lane, as the cooperative kernel) for finalize_tasks_kernel.
template <int BLOCK, int NB>
__global__ __launch_bounds__(BLOCK) void lsm_date_final_kernel(DevOpt o, const float* __restrict__ xs,
                                                               const float* __restrict__ vs,
                                                               const float* __restrict__ beta32,
                                                               const float* __restrict__ wcash,
                                                               int32_t* __restrict__ tau,
                                                               double* __restrict__ partials) {
  __shared__ double s_red[2 * (BLOCK / kWave)];
  const uint32_t p = blockIdx.x * BLOCK + threadIdx.x;
  const int N = o.steps;
  Kahan k1, k2;
  if (p < (uint32_t)o.paths) {
    float w;
    int32_t t = N;
    if (N == 1) {
      w = intrinsic(o, asset(o, xs[p])) * discount(o, 1);
    } else {
      w = wcash[p];
      t = tau[p];
      lsm_date_exercise<NB>(o, 1, xs[p], vs[p], beta32 + LsmLayout<NB>::kXW, w, t);
    }
    tau[p] = t;
    k1.add(w);
    k2.add(w * w);
  }
  double vals[2] = {k1.value(), k2.value()};
  block_sum<BLOCK, 2, double>(vals, s_red);
  if (threadIdx.x == 0) {
    partials[2 * (size_t)blockIdx.x] = vals[0];
    partials[2 * (size_t)blockIdx.x + 1] = vals[1];
  }
}

// Block t: the block partials of task t summed in block order (FP64), as finalize_rows_kernel,
// and the task's flags (block 0 also the launch status) copied after the sums.
__global__ __launch_bounds__(256) void finalize_tasks_kernel(const LsmTask* __restrict__ tasks,
                                                             const int32_t* __restrict__ status,
                                                             double* __restrict__ out) {
  __shared__ double s[256];
  const LsmTask& T = tasks[blockIdx.x];
  int32_t* fl = (int32_t*)(out + 2 * (size_t)gridDim.x);
  if (threadIdx.x == 0) {
    fl[blockIdx.x] = *T.flags;
    if (blockIdx.x == 0) fl[gridDim.x] = *status;
  }
  for (int32_t c = 0; c < 2; ++c) {
    double acc = 0.0;
    for (int32_t r = threadIdx.x; r < T.nblocks; r += 256) acc += T.partials[(size_t)r * 2 + c];
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
      if ((int)threadIdx.x < w) s[threadIdx.x] += s[threadIdx.x + w];
      __syncthreads();
    }
    if (threadIdx.x == 0) out[(size_t)blockIdx.x * 2 + c] = s[0];
    __syncthreads();
  }
}

// Exercise at t_1, then the discounted cash flow X = e^{-r tau dt} h of every path, summed per
// block (Kahan in FP32 per lane, FP64 across lanes) into tile partials {sum X, sum X^2}.
template <int BLOCK>
__global__ __launch_bounds__(BLOCK) void lsm_final_kernel(DevOpt o, const float* __restrict__ xs,
                                                          const float* __restrict__ vs,
                                                          float* __restrict__ hcash, int32_t* __restrict__ tau,
                                                          LsmState st, double* __restrict__ partials) {
  __shared__ double s_red[2 * (BLOCK / kWave)];
  const uint32_t p = blockIdx.x * BLOCK + threadIdx.x;
  const bool live = p < (uint32_t)o.paths;
  Kahan k1, k2;
  if (live) {
    float h_c = hcash[p];
    int32_t t = tau[p];
    if (o.steps > 1) {
      const float* b32 = st.beta32 + 8;
      if (b32[6] != 0.0f) {
        const int32_t t0 = t;
        lsm_exercise(o, b32, 1, xs[p], vs[p], h_c, t);
        if (t != t0) { hcash[p] = h_c; tau[p] = t; }
      }
    }
    const float X = h_c * discount(o, t);
    k1.add(X);
    k2.add(X * X);
  }
  double vals[2] = {k1.value(), k2.value()};
  block_sum<BLOCK, 2, double>(vals, s_red);
  if (threadIdx.x == 0) {
    partials[2 * (size_t)blockIdx.x] = vals[0];
    partials[2 * (size_t)blockIdx.x + 1] = vals[1];
  }
}

// ---------------------------------------------------------------------------------------------
// Greeks: forward pass with variance checkpoints, then the adjoint (reverse) sweep.
// ---------------------------------------------------------------------------------------------

// European forward pass for the Greeks: the payoff sums (as the pricing kernel, one path per
// lane) plus v at steps CK, 2 CK, ... (ck[(k - 1) * P + p]) and x_N (xN[p]).
template <int BLOCK, int SCHEME>
__global__ __launch_bounds__(BLOCK) void forward_ckpt_kernel(DevOpt o, int32_t CK, float* __restrict__ ck,
                                                             float* __restrict__ xN, double* __restrict__ partials) {
  __shared__ double s_red[2 * (BLOCK / kWave)];
  const uint32_t p = blockIdx.x * BLOCK + threadIdx.x;
  const bool live = p < (uint32_t)o.paths;
  const size_t P = (size_t)o.paths;
  float x = 0.0f, v = o.v0;
  for (int32_t n = 0; n < o.steps; ++n) {
    if (n > 0 && n % CK == 0 && live) ck[(size_t)(n / CK - 1) * P + p] = v;
    const Draw d = draw(o, (uint32_t)n, p);
    transition<SCHEME>(o, x, v, d);
  }
  Kahan k1, k2;
  if (live) {
    xN[p] = x;
    const float X = o.disc * intrinsic(o, asset(o, x));
    k1.add(X);
    k2.add(X * X);
  }
  double vals[2] = {k1.value(), k2.value()};
  block_sum<BLOCK, 2, double>(vals, s_red);
  if (threadIdx.x == 0) {
    partials[2 * (size_t)blockIdx.x] = vals[0];
    partials[2 * (size_t)blockIdx.x + 1] = vals[1];
  }
}

// Adjoint of one QE transition (v, V = v_{n+1}) given the running adjoint of V.  MG: Andersen's
// martingale-corrected step, whose constant is c0 = r dt - K13 v - g(A, m, s2) where the moment
// g = ln E[exp(A V) | v] exists (the steps the forward pass marks ok) and C0 elsewhere.
struct QEAdj {
  float E, A1, A2, Th;   // adjoints of the variance-step constants (Th: theta inside m)
  float K1, K2, K3, K4;  // adjoints of the log-price coefficients
  float rdt, C0, K13, Amg;  // MG: adjoints of r dt and C0 (their steps), of K13 and of A
};

// Adjoint of the truncated Gaussian variance step V = max(m (fm + fs Z1), 0), fm = mu / m and
// fs = sigma / m read from the table at l = log2(psi) as the forward step reads them: given Vbar,
// the adjoints of m and s2.  The derivatives of fm and log2 fs in l come from the table's second
// half (exact at the nodes, interpolated like the values); below the table fs = sqrt(psi) and
// fm = 1; above it the last entry holds (derivative 0); a truncated step (V = 0) passes nothing.
__device__ __forceinline__ void tg_variance_reverse(const DevOpt& o, float m, float s2, float z1, float Vbar,
                                                    float& mbar, float& s2bar) {
  mbar = 0.0f;
  s2bar = 0.0f;
  const float m2 = m * m;
  const float psi = s2 * rcp(m2);
  const float lp = __builtin_amdgcn_logf(psi);  // log2
  float fm, fs, dfm = 0.0f, dls = 0.0f;
  bool below = false, flat = false;
  if (lp < kTgLo) {
    below = true;
    fm = 1.0f;
    fs = fsqrt(psi);
  } else {
    const float traw = (lp - kTgLo) * kTgInvH;
    flat = traw > (float)(kTgN - 1);
    const float t = fminf(traw, (float)(kTgN - 1));
    const int i = min((int)t, kTgN - 2);
    const float f = t - (float)i;
    const float2 a = o.tg[i], b = o.tg[i + 1];
    fm = __builtin_fmaf(f, b.x - a.x, a.x);
    fs = __builtin_amdgcn_exp2f(__builtin_fmaf(f, b.y - a.y, a.y));
    const float2 da = o.tg[kTgN + i], db = o.tg[kTgN + i + 1];
    dfm = __builtin_fmaf(f, db.x - da.x, da.x);
    dls = __builtin_fmaf(f, db.y - da.y, da.y);
  }
  const float g = __builtin_fmaf(fs, z1, fm);
  if (!(m * g > 0.0f)) return;  // truncated at zero
  mbar = Vbar * g;
  const float gbar = Vbar * m;
  float psibar = 0.0f;
  if (below) {
    psibar = gbar * z1 * 0.5f * rcp(fs);  // d sqrt(psi) / d psi
  } else if (!flat) {
    // dg/dpsi = (dfm/dl + Z1 fs ln2 dls/dl) / (psi ln2)
    constexpr float kInvLn2 = 1.44269504088896340736f;
    const float ipsi = rcp(psi);
    psibar = gbar * __builtin_fmaf(dfm * kInvLn2, ipsi, z1 * fs * dls * ipsi);
  }
  s2bar = psibar * rcp(m2);
  mbar -= 2.0f * psibar * psi * rcp(m);
}

// KIND 0: QE; 1: martingale-corrected QE; 2: truncated Gaussian variance with QE's log-price step.
template <int KIND>
__device__ __forceinline__ float qe_reverse(const DevOpt& o, float v, float V, float z1, float z2, float u,
                                            float xbar, float vbar_next, QEAdj& a) {
  constexpr bool MG = KIND == 1;
  // log-price step: x' = x + c0 + K1 v + K2 V + sqrt(K3 v + K4 V) Z2
  const float w = __builtin_fmaf(o.K3, v, o.K4 * V);
  const float sw = fsqrt(w);
  const float q = (sw > 0.0f) ? xbar * z2 * 0.5f * rcp(sw) : 0.0f;
  a.K1 = __builtin_fmaf(xbar, v, a.K1);
  a.K2 = __builtin_fmaf(xbar, V, a.K2);
  a.K3 = __builtin_fmaf(q, v, a.K3);
  a.K4 = __builtin_fmaf(q, V, a.K4);
  const float Vbar = vbar_next + xbar * o.K2 + q * o.K4;
  float vbar = xbar * o.K1 + q * o.K3;
  // variance step, recomputed (psi exactly as the forward step forms it, so the branch is the same)
  const float m = __builtin_fmaf(v - o.theta, o.E, o.theta);
  const float s2 = __builtin_fmaf(v, o.A1, o.A2);
  const float A = o.Amg;
  const float gbar = -xbar;  // MG, ok steps: d c0 / d g = -1
  bool ok = true;
  float mbar = 0.0f, s2bar = 0.0f;
  if (!(s2 > 0.0f)) {
    mbar = Vbar;
    if constexpr (MG) {  // g = A m
      a.Amg = __builtin_fmaf(gbar, m, a.Amg);
      mbar = __builtin_fmaf(gbar, A, mbar);
    }
  } else if constexpr (KIND == 2) {
    tg_variance_reverse(o, m, s2, z1, Vbar, mbar, s2bar);
  } else {
    const float m2 = m * m;
    const float rm = rcp(m);
    const float psi = s2 * rcp(m2);
    float psibar = 0.0f;
    if (psi <= kPsiC) {
      const float t = 2.0f * m2 * rcp(s2);
      const float rt = fsqrt(t * (t - 1.0f));
      const float b2 = (t - 1.0f) + rt;
      const float b = fsqrt(b2);
      const float ib = rcp(1.0f + b2);
      const float a_ = m * ib;
      const float bz = b + z1;
      float abar = Vbar * bz * bz;
      const float bbar = Vbar * 2.0f * a_ * bz;
      float b2bar = bbar * 0.5f * rcp(b);
      if constexpr (MG) {
        // g = A b2 a / dd - ln(dd) / 2, dd = 1 - 2 A a:
        // dg/da = (A / dd) f, dg/dA = (a / dd) f with f = 1 + b2 (1 + 2 A a / dd); dg/db2 = A a / dd
        const float dd = __builtin_fmaf(-2.0f * A, a_, 1.0f);
        ok = dd > 0.0f;
        if (ok) {
          const float idd = rcp(dd);
          const float f = __builtin_fmaf(b2, __builtin_fmaf(2.0f * A * a_, idd, 1.0f), 1.0f);
          const float ga = gbar * idd;
          abar = __builtin_fmaf(ga * A, f, abar);
          b2bar = __builtin_fmaf(ga * A, a_, b2bar);
          a.Amg = __builtin_fmaf(ga * a_, f, a.Amg);
        }
      }
      mbar = abar * ib;
      b2bar = __builtin_fmaf(-abar * a_, ib, b2bar);
      const float tbar = b2bar * (1.0f + (2.0f * t - 1.0f) * 0.5f * rcp(rt));
      psibar = -tbar * t * t * 0.5f;
    } else {
      const float p = (psi - 1.0f) * rcp(psi + 1.0f);
      const float omp = 1.0f - p;
      float pbar = 0.0f;
      if (u > p) {
        const float iomp = rcp(omp);
        const float L = __builtin_amdgcn_logf(omp * rcp(1.0f - u)) * 0.69314718055994530942f;
        mbar = Vbar * L * iomp;
        pbar = Vbar * m * (L - 1.0f) * iomp * iomp;
      }
      if constexpr (MG) {
        // g = ln G, G = p + beta (1 - p) / (beta - A), beta = (1 - p) / m:
        // dG/dp = 1 - beta / (beta - A), dG/dbeta = -A (1 - p) / (beta - A)^2, dG/dA = beta (1 - p) / (beta - A)^2
        const float beta = omp * rcp(m);
        ok = A < beta;
        if (ok) {
          const float ibA = rcp(beta - A);
          const float gG = gbar * rcp(__builtin_fmaf(beta * omp, ibA, p));
          const float qq = gG * omp * ibA * ibA;
          pbar = __builtin_fmaf(gG, __builtin_fmaf(-beta, ibA, 1.0f), pbar);
          a.Amg = __builtin_fmaf(qq, beta, a.Amg);
          const float betabar = -qq * A;
          pbar = __builtin_fmaf(-betabar, rm, pbar);
          mbar = __builtin_fmaf(-betabar * beta, rm, mbar);
        }
      }
      const float ip1 = rcp(psi + 1.0f);
      psibar = pbar * 2.0f * ip1 * ip1;
    }
    s2bar = psibar * rm * rm;
    mbar -= 2.0f * psibar * psi * rm;
  }
  if constexpr (MG) {
    if (ok) {
      a.rdt += xbar;
      a.K13 = __builtin_fmaf(-xbar, v, a.K13);
      vbar = __builtin_fmaf(-xbar, o.K13, vbar);
    } else {
      a.C0 += xbar;
    }
  }
  a.Th = __builtin_fmaf(mbar, 1.0f - o.E, a.Th);
  a.E = __builtin_fmaf(mbar, v - o.theta, a.E);
  a.A1 = __builtin_fmaf(s2bar, v, a.A1);
  a.A2 += s2bar;
  vbar = __builtin_fmaf(mbar, o.E, vbar);
  vbar = __builtin_fmaf(s2bar, o.A1, vbar);
  return vbar;
}

// Adjoint of one full-truncation Euler transition: x' = x + rdt - hdt v+ + sdt sqrt(v+) zs,
// v' = v + kthdt - kdt v+ + xisdt sqrt(v+) z1, zs = rho z1 + srho z2, v+ = max(v, 0); the
// derivative of sqrt at 0 (and of srho at |rho| = 1) is taken as 0.  Accumulates the
// constants' adjoints and returns the adjoint of v.
struct FTEAdj {
  float rdt, hdt, sdt, rho, kthdt, kdt, xisdt;
};

__device__ __forceinline__ float fte_reverse(const DevOpt& o, float v, float z1, float z2, float xbar,
                                             float vbar_next, FTEAdj& a) {
  const float vp = fmaxf(v, 0.0f);
  const float sv = fsqrt(vp);
  const float zs = __builtin_fmaf(o.rho, z1, o.srho * z2);
  a.rdt += xbar;
  a.hdt = __builtin_fmaf(-xbar, vp, a.hdt);
  a.sdt = __builtin_fmaf(xbar * sv, zs, a.sdt);
  const float dzs = (o.srho > 0.0f) ? z1 - o.rho * rcp(o.srho) * z2 : z1;  // d zs / d rho
  a.rho = __builtin_fmaf(xbar * o.sdt * sv, dzs, a.rho);
  a.kthdt += vbar_next;
  a.kdt = __builtin_fmaf(-vbar_next, vp, a.kdt);
  a.xisdt = __builtin_fmaf(vbar_next * sv, z1, a.xisdt);
  float vbar = vbar_next;
  if (v > 0.0f) {
    const float isv = (sv > 0.0f) ? 0.5f * rcp(sv) : 0.0f;
    const float dx = __builtin_fmaf(o.sdt * zs, isv, -o.hdt);   // d x' / d v+
    const float dv = __builtin_fmaf(o.xisdt * z1, isv, -o.kdt);  // d (v' - v) / d v+
    vbar = __builtin_fmaf(vbar_next, dv, vbar_next) + xbar * dx;
  }
  return vbar;
}

// Reverse sweep, one path per lane.  Path p stops at tau_p (N for European options, the
// Longstaff-Schwartz exercise index for American ones, held fixed); its discounted cash flow is
// X = e^{-r tau dt} h(S0 e^{x_tau}).  The sweep walks the segments [k CK, (k+1) CK) from the
// last one down: it recomputes the segment forward from the variance checkpoint v_{k CK}
// (regenerating the counter-based random numbers, so the draws are the forward pass's bit for
// bit), keeps the segment in registers, and runs the reverse transitions.  The 7 Greeks of
// the path follow from the step-constant adjoints by the chain rule, and their sums and sums of
// squares (Kahan FP32 per lane, FP64 across the block) go to one row of 14 doubles per block.
// The reverse sweep of every path of a block.  A wave runs as long as its longest path and only
// paths with a positive stopped payoff contribute, so the block first orders its paths by exercise
// index in classes of 8 steps, longest first (ncls = min(ceil(N / 8), kAdjClasses) classes, the
// first also taking anything longer), the out-of-the-money ones last: a stable counting sort in
// LDS (lane rank by wave ballots, per-wave class counts, prefixes over waves and classes), so the
// order -- and every sum over it -- is deterministic and does not depend on the checkpoint
// interval.  Thread t then sweeps the path at sorted position t.
// EXT adds d/dT (steps fixed; the adjoints of the step constants times their T-derivatives, and
// the discount) and, for European options, gamma by the pathwise likelihood-ratio estimator:
// conditional on the variance path x_tau is Gaussian in the asset variates z2_n with variance
// sum sigma_n^2 (sigma_n = sqrt(K3 v_n + K4 v_{n+1})), so with W = sum sigma_n z2_n / sum sigma_n^2
// and xbar = dX / d ln S0 the path's term is xbar (W - 1) / S0^2 (NaN if sum sigma_n^2 = 0; NaN
// for American options, whose stopping decisions would be re-weighted onto other paths).
// gpartials: 2 NG doubles per block (sums, then sums of squares), NG = 7 or 9.
template <int BLOCK, int CK, bool EXT, int SCHEME>
__global__ __launch_bounds__(BLOCK) void adjoint_kernel(DevOpt o, const float* __restrict__ ck_base,
                                                        size_t ck_stride, const float* __restrict__ xstop,
                                                        const int32_t* __restrict__ tau,
                                                        double* __restrict__ gpartials) {
  constexpr int W = BLOCK / kWave;
  constexpr int NG = EXT ? 9 : 7;
  __shared__ double s_red[2 * NG * W];
  __shared__ uint16_t s_cnt[W][kAdjClasses + 1];
  __shared__ uint16_t s_base[kAdjClasses + 1];
  __shared__ uint16_t s_slot[BLOCK];
  __shared__ int32_t s_ts[BLOCK];
  __shared__ float s_xs[BLOCK];
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  const size_t P = (size_t)o.paths;
  const int ncls = min((o.steps + 7) / 8, kAdjClasses);
  {
    const uint32_t p = blockIdx.x * BLOCK + threadIdx.x;
    int32_t ts = 0;  // 0: nothing to sweep
    float xs = 0.0f;
    int c = ncls;
    if (p < (uint32_t)o.paths) {
      ts = tau ? tau[p] : o.steps;
      if (ts >= 1 && ts <= o.steps) {
        xs = tau ? xstop[(size_t)(ts - 1) * P + p] : xstop[p];
        if (intrinsic(o, asset(o, xs)) > 0.0f) c = ncls - min((ts + 7) / 8, ncls);
      } else {
        ts = 0;
      }
    }
    s_ts[threadIdx.x] = ts;
    s_xs[threadIdx.x] = xs;
    for (int i = threadIdx.x; i < W * (kAdjClasses + 1); i += BLOCK) (&s_cnt[0][0])[i] = 0;
    __syncthreads();
    const uint64_t lt = lane ? (~0ull >> (kWave - lane)) : 0ull;
    uint64_t todo = ~0ull;
    int rank = 0;
    while (todo) {  // one ballot per class present in the wave
      const int leader = __builtin_ctzll(todo);
      const int c0 = __shfl(c, leader, kWave);
      const uint64_t m = __ballot(c == c0);
      if (c == c0) rank = __popcll(m & lt);
      if (lane == leader) s_cnt[wid][c0] = (uint16_t)__popcll(m);
      todo &= ~m;
    }
    __syncthreads();
    if ((int)threadIdx.x <= ncls) {  // thread j: prefix of class j over the waves, and its total
      uint16_t run = 0;
      for (int w = 0; w < W; ++w) {
        const uint16_t v = s_cnt[w][threadIdx.x];
        s_cnt[w][threadIdx.x] = run;
        run += v;
      }
      s_base[threadIdx.x] = run;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      uint16_t run = 0;
      for (int j = 0; j <= ncls; ++j) {
        const uint16_t v = s_base[j];
        s_base[j] = run;
        run += v;
      }
    }
    __syncthreads();
    s_slot[s_base[c] + s_cnt[wid][c] + rank] = (uint16_t)threadIdx.x;
    __syncthreads();
  }
  const int src = s_slot[threadIdx.x];
  const uint32_t p = blockIdx.x * BLOCK + (uint32_t)src;
  const int32_t ts = s_ts[src];
  float g[NG];
#pragma unroll
  for (int i = 0; i < NG; ++i) g[i] = 0.0f;
  if (ts > 0) {
    const float xs = s_xs[src];
    const float S = asset(o, xs);
    const float h = intrinsic(o, S);
    const float D = discount(o, ts);
    if (h > 0.0f) {
      const float xbar = D * S * (is_call(o.payoff) ? 1.0f : -1.0f);  // dX/dx_tau
      QEAdj a = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
      FTEAdj af = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
      float vbar = 0.0f;
      float sz = 0.0f, ss = 0.0f;  // gamma: sum sigma_n z2_n, sum sigma_n^2
      const int32_t nseg = (ts + CK - 1) / CK;
      for (int32_t k = nseg - 1; k >= 0; --k) {
        const int32_t start = k * CK;
        const int32_t len = min(CK, ts - start);
        float vv[CK + 1], z1[CK], z2[CK], uu[CK];
        vv[0] = (k == 0) ? o.v0 : ck_base[(size_t)(k - 1) * ck_stride + p];
        // the segment's draws first (independent of each other and of the state, so they
        // overlap freely; past the stop they are unused), then the variance chain
#pragma unroll
        for (int i = 0; i < CK; ++i) {
          const Draw d = draw(o, (uint32_t)(start + i), p);
          z1[i] = d.z1;
          z2[i] = d.z2;
          uu[i] = d.u;
        }
#pragma unroll
        for (int i = 0; i < CK; ++i) {
          if (i < len) {
            if constexpr (SCHEME == 3) vv[i + 1] = tg_variance(o, vv[i], z1[i]);
            else if constexpr (SCHEME != 1) vv[i + 1] = qe_variance(o, vv[i], z1[i], uu[i]);
            else vv[i + 1] = fte_variance(o, vv[i], z1[i]);
            if constexpr (EXT) {  // the coefficient of z2 in the log-price step
              const float sig = SCHEME != 1 ? fsqrt(__builtin_fmaf(o.K3, vv[i], o.K4 * vv[i + 1]))
                                            : o.sdt * fsqrt(fmaxf(vv[i], 0.0f)) * o.srho;
              sz = __builtin_fmaf(sig, z2[i], sz);
              ss = __builtin_fmaf(sig, sig, ss);
            }
          }
        }
#pragma unroll
        for (int i = CK - 1; i >= 0; --i) {
          if (i < len) {
            if constexpr (SCHEME != 1)
              vbar = qe_reverse<SCHEME == 2 ? 1 : (SCHEME == 3 ? 2 : 0)>(o, vv[i], vv[i + 1], z1[i], z2[i], uu[i],
                                                                      xbar, vbar, a);
            else vbar = fte_reverse(o, vv[i], z1[i], z2[i], xbar, vbar, af);
          }
        }
      }
      const float X = D * h;
      g[0] = xbar / o.S0;
      g[1] = vbar;
      if constexpr (SCHEME != 1) {
        // QE: C0 on every step.  Martingale-corrected QE: C0 on the steps without the moment,
        // r dt on the others, and K13 = K1 + K3 / 2, A = K2 + K4 / 2 folded into K1..K4.
        const float aC0 = SCHEME == 2 ? a.C0 : (float)ts * xbar;
        const float aR = SCHEME == 2 ? a.rdt : 0.0f;
        float k1 = a.K1, k2 = a.K2, k3 = a.K3, k4 = a.K4;
        if constexpr (SCHEME == 2) {
          k1 += a.K13;
          k2 += a.Amg;
          k3 = __builtin_fmaf(0.5f, a.K13, k3);
          k4 = __builtin_fmaf(0.5f, a.Amg, k4);
        }
        g[2] = a.Th + a.A2 * o.dA2_dth + aC0 * o.dC0_dth;
        g[3] = -(float)ts * o.dt * X + aC0 * o.dC0_dr + aR * o.dt;
        g[4] = a.E * o.dE_dk + a.A1 * o.dA1_dk + a.A2 * o.dA2_dk + aC0 * o.dC0_dk + k1 * o.dK1_dk + k2 * o.dK2_dk;
        g[5] = a.A1 * o.dA1_dxi + a.A2 * o.dA2_dxi + aC0 * o.dC0_dxi + k1 * o.dK1_dxi + k2 * o.dK2_dxi;
        g[6] = aC0 * o.dC0_drho + k1 * o.dK1_drho + k2 * o.dK2_drho + k3 * o.dK3_drho + k4 * o.dK4_drho;
        if constexpr (EXT)
          g[7] = a.E * o.dE_dT + a.A1 * o.dA1_dT + a.A2 * o.dA2_dT + aC0 * o.dC0_dT + (k1 * o.dK1_dT + k2 * o.dK2_dT) +
                 (k3 + k4) * o.dK3_dT + aR * o.rN - (float)ts * o.rN * X;
      } else {
        // kdt = kappa dt, kthdt = kappa theta dt, xisdt = xi sqrt(dt), rdt = r dt
        g[2] = af.kthdt * o.kdt;
        g[3] = af.rdt * o.dt - (float)ts * o.dt * X;
        g[4] = af.kdt * o.dt + af.kthdt * o.theta * o.dt;
        g[5] = af.xisdt * o.sdt;
        g[6] = af.rho;
        if constexpr (EXT)
          g[7] = af.rdt * o.fdT_rdt + af.hdt * o.fdT_hdt + af.sdt * o.fdT_sdt + af.kdt * o.fdT_kdt +
                 af.kthdt * o.fdT_kthdt + af.xisdt * o.fdT_xisdt - (float)ts * o.rN * X;
      }
      if constexpr (EXT) {
        g[8] = tau ? __builtin_nanf("") : (ss > 0.0f ? xbar * (sz / ss - 1.0f) / (o.S0 * o.S0) : __builtin_nanf(""));
      }
    }
  }
  double vals[2 * NG];
#pragma unroll
  for (int i = 0; i < NG; ++i) {
    Kahan s, s2;
    s.add(g[i]);
    s2.add(g[i] * g[i]);
    vals[i] = s.value();
    vals[NG + i] = s2.value();
  }
  block_sum<BLOCK, 2 * NG, double>(vals, s_red);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < 2 * NG; ++i) gpartials[(size_t)blockIdx.x * 2 * NG + i] = vals[i];
  }
}

// ---------------------------------------------------------------------------------------------
// Debug dumps.
// ---------------------------------------------------------------------------------------------
__global__ void debug_draws_kernel(uint32_t seed_lo, uint32_t seed_hi, uint32_t stream, int64_t path0,
                                   int64_t npaths, int32_t step0, int32_t nsteps, uint32_t* __restrict__ words,
                                   float* __restrict__ unif, float* __restrict__ norm) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= npaths * nsteps) return;
  const int64_t pi = e / nsteps;
  const int32_t ni = (int32_t)(e - pi * nsteps);
  const Words w = philox4x32_10((uint32_t)(step0 + ni), (uint32_t)(path0 + pi), stream, 0u, seed_lo, seed_hi);
  if (words) {
    words[4 * e] = w.w0;
    words[4 * e + 1] = w.w1;
    words[4 * e + 2] = w.w2;
    words[4 * e + 3] = w.w3;
  }
  const float u0 = u01(w.w0), u1 = u01(w.w1), u2 = u01(w.w2);
  if (unif) {
    unif[3 * e] = u0;
    unif[3 * e + 1] = u1;
    unif[3 * e + 2] = u2;
  }
  if (norm) {
    float z1, z2;
    box_muller(u0, u1, z1, z2);
    norm[2 * e] = z1;
    norm[2 * e + 1] = z2;
  }
}

template <int SCHEME>
__global__ __launch_bounds__(256) void debug_paths_kernel(DevOpt o, float* __restrict__ xT, float* __restrict__ vT,
                                                          float* __restrict__ pay) {
  const uint32_t p = blockIdx.x * 256 + threadIdx.x;
  if (p >= (uint32_t)o.paths) return;
  float x = 0.0f, v = o.v0;
  for (int32_t n = 0; n < o.steps; ++n) {
    const Draw d = draw(o, (uint32_t)n, p);
    transition<SCHEME>(o, x, v, d);
  }
  if (xT) xT[p] = x;
  if (vT) vT[p] = v;
  if (pay) pay[p] = o.disc * intrinsic(o, asset(o, x));
}

// ---------------------------------------------------------------------------------------------
// Host-side launchers.
// ---------------------------------------------------------------------------------------------
template <int SCHEME, int BLOCK, int PPL>
static hipError_t launch_batch_t(const BatchLaunch& L, hipStream_t s) {
  hipLaunchKernelGGL((batch_price_kernel<SCHEME, BLOCK, PPL>), dim3(L.grid), dim3(BLOCK), 0, s, L.opts, L.order,
                     L.uprefix, L.nopt, L.nunits, L.counter, L.partials);
  return hipGetLastError();
}

template <int SCHEME>
static hipError_t launch_batch_s(const BatchLaunch& L, hipStream_t s) {
  switch (L.block * 8 + L.ppl) {
    case 128 * 8 + 1: return launch_batch_t<SCHEME, 128, 1>(L, s);
    case 128 * 8 + 2: return launch_batch_t<SCHEME, 128, 2>(L, s);
    case 128 * 8 + 4: return launch_batch_t<SCHEME, 128, 4>(L, s);
    case 256 * 8 + 1: return launch_batch_t<SCHEME, 256, 1>(L, s);
    case 256 * 8 + 2: return launch_batch_t<SCHEME, 256, 2>(L, s);
    case 256 * 8 + 4: return launch_batch_t<SCHEME, 256, 4>(L, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_batch_price(int scheme, const BatchLaunch& L, hipStream_t s) {
  if (scheme == 0) return launch_batch_s<0>(L, s);
  if (scheme == 1) return launch_batch_s<1>(L, s);
  if (scheme == 2) return launch_batch_s<2>(L, s);
  if (scheme == 3) return launch_batch_s<3>(L, s);
  if (scheme == 4) return launch_batch_s<4>(L, s);
  return hipErrorInvalidValue;
}

int batch_kernel_occupancy(int scheme, int block, int ppl) {
  int nb = 0;
  hipError_t e = hipErrorInvalidValue;
#define SIMR_OCC(S, B, Q) \
  if (scheme == S && block == B && ppl == Q) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, batch_price_kernel<S, B, Q>, B, 0);
  SIMR_OCC(0, 128, 1) SIMR_OCC(0, 128, 2) SIMR_OCC(0, 128, 4) SIMR_OCC(0, 256, 1) SIMR_OCC(0, 256, 2) SIMR_OCC(0, 256, 4)
  SIMR_OCC(1, 128, 1) SIMR_OCC(1, 128, 2) SIMR_OCC(1, 128, 4) SIMR_OCC(1, 256, 1) SIMR_OCC(1, 256, 2) SIMR_OCC(1, 256, 4)
  SIMR_OCC(2, 128, 1) SIMR_OCC(2, 128, 2) SIMR_OCC(2, 128, 4) SIMR_OCC(2, 256, 1) SIMR_OCC(2, 256, 2) SIMR_OCC(2, 256, 4)
  SIMR_OCC(3, 128, 1) SIMR_OCC(3, 128, 2) SIMR_OCC(3, 128, 4) SIMR_OCC(3, 256, 1) SIMR_OCC(3, 256, 2) SIMR_OCC(3, 256, 4)
  SIMR_OCC(4, 128, 1) SIMR_OCC(4, 128, 2) SIMR_OCC(4, 128, 4) SIMR_OCC(4, 256, 1) SIMR_OCC(4, 256, 2) SIMR_OCC(4, 256, 4)
#undef SIMR_OCC
  return e == hipSuccess ? nb : 0;
}

hipError_t launch_finalize_rows(const double* rows, int ncol, const DevOpt* opts, int nopt, int nrows, double* out,
                                hipStream_t s) {
  hipLaunchKernelGGL(finalize_rows_kernel, dim3(opts ? nopt : ncol), dim3(256), 0, s, rows, ncol, opts, nrows, out);
  return hipGetLastError();
}

hipError_t launch_reset_words(uint32_t* p, int64_t n, hipStream_t s) {
  const int64_t blocks = std::min<int64_t>(std::max<int64_t>((n + 4095) / 4096, 1), 1024);
  hipLaunchKernelGGL(reset_words_kernel, dim3((unsigned)blocks), dim3(256), 0, s, p, n);
  return hipGetLastError();
}

hipError_t launch_forward_spill(int scheme, const DevOpt& o, float* xs, float* vs, uint32_t* zero, int64_t nzero,
                                hipStream_t s) {
  const int grid = (o.paths + kLsmBlock - 1) / kLsmBlock;
  if (scheme == 0)
    hipLaunchKernelGGL((forward_spill_kernel<0, kLsmBlock>), dim3(grid), dim3(kLsmBlock), 0, s, o, xs, vs, zero, nzero);
  else if (scheme == 1)
    hipLaunchKernelGGL((forward_spill_kernel<1, kLsmBlock>), dim3(grid), dim3(kLsmBlock), 0, s, o, xs, vs, zero, nzero);
  else if (scheme == 2)
    hipLaunchKernelGGL((forward_spill_kernel<2, kLsmBlock>), dim3(grid), dim3(kLsmBlock), 0, s, o, xs, vs, zero, nzero);
  else if (scheme == 3)
    hipLaunchKernelGGL((forward_spill_kernel<3, kLsmBlock>), dim3(grid), dim3(kLsmBlock), 0, s, o, xs, vs, zero, nzero);
  else if (scheme == 4)
    hipLaunchKernelGGL((forward_spill_kernel<4, kLsmBlock>), dim3(grid), dim3(kLsmBlock), 0, s, o, xs, vs, zero, nzero);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_lsm(const DevOpt& o, const float* xs, const float* vs, float* hcash, int32_t* tau,
                      const LsmState& st, double* partials, hipStream_t s) {
  const int grid = (o.paths + kLsmBlock - 1) / kLsmBlock;
  hipLaunchKernelGGL((lsm_init_kernel<kLsmBlock>), dim3(grid), dim3(kLsmBlock), 0, s, o, xs, hcash, tau);
  for (int32_t n = o.steps - 1; n >= 1; --n)
    hipLaunchKernelGGL((lsm_step_kernel<kLsmBlock>), dim3(grid), dim3(kLsmBlock), 0, s, o, n, xs, vs, hcash, tau, st);
  hipLaunchKernelGGL((lsm_final_kernel<kLsmBlock>), dim3(grid), dim3(kLsmBlock), 0, s, o, xs, vs, hcash, tau, st,
                     partials);
  return hipGetLastError();
}

template <int BLOCK, int PPL, int NB>
static int lsm_coop_capacity() {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, lsm_persistent_kernel<BLOCK, PPL, NB>, BLOCK, 0) !=
      hipSuccess)
    return 0;
  return nb;
}

template <int BLOCK, int PPL, int NB>
static hipError_t launch_lsm_coop_t(const LsmTask* tasks, int ntasks, int grid, int32_t* status, hipStream_t s) {
  const LsmTask* a0 = tasks;
  int32_t a1 = ntasks;
  int32_t* a2 = status;
  void* args[] = {&a0, &a1, &a2};
  return hipLaunchCooperativeKernel((const void*)lsm_persistent_kernel<BLOCK, PPL, NB>, dim3(grid), dim3(BLOCK), args,
                                    0, s);
}

// Shapes of the cooperative induction: an option's paths per block, kLsmVBlock x 1, 2 or 4
// (most latency-tolerant first: fewer paths per lane, more waves per CU), fix its grid and its
// bits.  A launch runs them on 1024-thread blocks, or on 256-thread blocks with 4x the paths
// per lane (the same bits), which fit more blocks per CU.  The 10-function basis keeps the
// 1024-thread blocks (its per-path basis values live in registers across the exchange).
static const int kCoopPpl[] = {1, 2, 4};
constexpr int kCoopShapes = 3;

static int coop_capacity(int block, int ppl, int nb) {
  if (nb == 10) {
    if (block == 1024 && ppl == 1) return lsm_coop_capacity<1024, 1, 10>();
    if (block == 1024 && ppl == 2) return lsm_coop_capacity<1024, 2, 10>();
    if (block == 1024 && ppl == 4) return lsm_coop_capacity<1024, 4, 10>();
    return 0;
  }
  if (block == 1024 && ppl == 1) return lsm_coop_capacity<1024, 1, 6>();
  if (block == 1024 && ppl == 2) return lsm_coop_capacity<1024, 2, 6>();
  if (block == 1024 && ppl == 4) return lsm_coop_capacity<1024, 4, 6>();
  if (block == 256 && ppl == 4) return lsm_coop_capacity<256, 4, 6>();
  if (block == 256 && ppl == 8) return lsm_coop_capacity<256, 8, 6>();
  if (block == 256 && ppl == 16) return lsm_coop_capacity<256, 16, 6>();
  return 0;
}

// Every option takes the shape it would take alone: the first whose grid fits within gmax
// blocks, else within 256.  Consecutive options of one shape then share launches while their
// blocks fit co-resident, on whichever block size holds more of them (1024 threads on a tie,
// or the size `block` names if nonzero and the option fits it).  An option's result therefore
// depends neither on the others nor on the block size.
std::vector<LsmLaunchSet> lsm_coop_plan(const std::vector<int64_t>& paths, int num_cus, int gmax,
                                        std::vector<int>* grids, int nb, int block) {
  if (nb != 6) block = 1024;
  int cap[2][kCoopShapes];  // co-resident blocks: [0] 1024 threads, [1] 256 threads
  for (int q = 0; q < kCoopShapes; ++q) {
    cap[0][q] = block == 256 ? 0 : coop_capacity(1024, kCoopPpl[q], nb) * num_cus;
    cap[1][q] = block == 1024 ? 0 : coop_capacity(256, 4 * kCoopPpl[q], nb) * num_cus;
  }
  const int n = (int)paths.size();
  grids->assign(n, 0);
  std::vector<int> shape(n, -1);
  for (int i = 0; i < n; ++i) {
    const int64_t caps[2] = {std::min(gmax, 256), 256};
    for (int pass = 0; pass < 2 && shape[i] < 0; ++pass)
      for (int q = 0; q < kCoopShapes && shape[i] < 0; ++q) {
        const int64_t per = (int64_t)kLsmVBlock * kCoopPpl[q];
        const int64_t g = (paths[i] + per - 1) / per;
        if (g <= std::min<int64_t>(std::max(cap[0][q], cap[1][q]), caps[pass])) {
          shape[i] = q;
          (*grids)[i] = (int)g;
        }
      }
    if (shape[i] < 0) return {};
  }
  std::vector<LsmLaunchSet> sets;
  for (int i = 0; i < n;) {
    const int q = shape[i];
    int count[2] = {0, 0}, grid[2] = {0, 0};
    for (int z = 0; z < 2; ++z)
      while (i + count[z] < n && shape[i + count[z]] == q && grid[z] + (*grids)[i + count[z]] <= cap[z][q]) {
        grid[z] += (*grids)[i + count[z]];
        ++count[z];
      }
    const int z = count[1] > count[0] ? 1 : 0;
    LsmLaunchSet ls{i, count[z], z ? 256 : 1024, z ? 4 * kCoopPpl[q] : kCoopPpl[q], grid[z]};
    sets.push_back(ls);
    i += count[z];
  }
  return sets;
}

// Gram sums of every date, then one factorisation per date.
hipError_t launch_lsm_gram(const DevOpt& o, const float* xs, const float* vs, float* gram, hipStream_t s, int nb) {
  if (o.steps < 2) return hipSuccess;
  const int chunks = lsm_gram_chunks(o.paths);
  const int per_lane = (int)((o.paths + (int64_t)chunks * kLsmBlock - 1) / ((int64_t)chunks * kLsmBlock));
  if (per_lane > kGramMaxPerLane) return hipErrorInvalidValue;  // the chunks are sized to keep it <= 16
  if (nb == 6) {
    hipLaunchKernelGGL((lsm_gram_kernel<kLsmBlock, 6>), dim3(o.steps - 1, chunks), dim3(kLsmBlock), 0, s, o, xs,
                       vs, per_lane, gram);
  } else if (nb == 10) {
    hipLaunchKernelGGL((lsm_gram_kernel<kLsmBlock, 10>), dim3(o.steps - 1, chunks), dim3(kLsmBlock), 0, s, o, xs,
                       vs, per_lane, gram);
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// The FP64 factorisations of every date's Gram sums (after launch_lsm_gram on the same stream).
hipError_t launch_lsm_factor(const DevOpt& o, double rdt, const float* gram, double* fac, int32_t* flags,
                             hipStream_t s, int nb) {
  if (o.steps < 2) return hipSuccess;
  const int chunks = lsm_gram_chunks(o.paths);
  if (nb == 6) {
    hipLaunchKernelGGL(lsm_factor_kernel, dim3(o.steps - 1), dim3(kFactorThreads), 0, s, chunks, rdt, gram, fac,
                       flags);
  } else if (nb == 10) {
    hipLaunchKernelGGL((lsm_factor_serial_kernel<10>), dim3(o.steps - 1), dim3(64), 0, s, chunks, rdt, gram, fac,
                       flags);
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// The cooperative induction over all dates of every task (factors from launch_lsm_factor).
hipError_t launch_lsm_coop(const LsmTask* tasks, int ntasks, int block, int ppl, int grid, int32_t* status,
                           hipStream_t s, int nb) {
  if (nb == 10) {
    if (block == 1024 && ppl == 1) return launch_lsm_coop_t<1024, 1, 10>(tasks, ntasks, grid, status, s);
    if (block == 1024 && ppl == 2) return launch_lsm_coop_t<1024, 2, 10>(tasks, ntasks, grid, status, s);
    if (block == 1024 && ppl == 4) return launch_lsm_coop_t<1024, 4, 10>(tasks, ntasks, grid, status, s);
    return hipErrorInvalidValue;
  }
  if (nb != 6) return hipErrorInvalidValue;
  if (block == 1024 && ppl == 1) return launch_lsm_coop_t<1024, 1, 6>(tasks, ntasks, grid, status, s);
  if (block == 1024 && ppl == 2) return launch_lsm_coop_t<1024, 2, 6>(tasks, ntasks, grid, status, s);
  if (block == 1024 && ppl == 4) return launch_lsm_coop_t<1024, 4, 6>(tasks, ntasks, grid, status, s);
  if (block == 256 && ppl == 4) return launch_lsm_coop_t<256, 4, 6>(tasks, ntasks, grid, status, s);
  if (block == 256 && ppl == 8) return launch_lsm_coop_t<256, 8, 6>(tasks, ntasks, grid, status, s);
  if (block == 256 && ppl == 16) return launch_lsm_coop_t<256, 16, 6>(tasks, ntasks, grid, status, s);
  return hipErrorInvalidValue;
}

hipError_t launch_stage_record(const void* src, size_t bytes, void* dst, hipStream_t s) {
  if (bytes > sizeof(Record1K) || bytes % 4 != 0 || !src || !dst) return hipErrorInvalidValue;
  Record1K r;
  std::memset(&r, 0, sizeof r);
  std::memcpy(&r, src, bytes);
  hipLaunchKernelGGL(stage_record_kernel, dim3(1), dim3(256), 0, s, r, (uint32_t)(bytes / 4), (uint32_t*)dst);
  return hipGetLastError();
}

hipError_t launch_finalize_tasks(const LsmTask* tasks, int ntasks, const int32_t* status, double* out,
                                 hipStream_t s) {
  hipLaunchKernelGGL(finalize_tasks_kernel, dim3(ntasks), dim3(256), 0, s, tasks, status, out);
  return hipGetLastError();
}

template <int NB>
static hipError_t launch_lsm_dates_t(const DevOpt& o, const float* xs, const float* vs, const double* fac,
                                     float* wcash, int32_t* tau, float* gpart, float* beta32, double* beta64,
                                     uint32_t* ticket, double* partials, hipStream_t s) {
  const int grid = (int)((o.paths + kLsmBlock - 1) / kLsmBlock);
  for (int32_t n = o.steps - 1; n >= 1; --n)
    hipLaunchKernelGGL((lsm_date_kernel<kLsmBlock, NB>), dim3(grid), dim3(kLsmBlock), 0, s, o, n, xs, vs, fac, wcash,
                       tau, gpart, beta32, beta64, ticket);
  hipLaunchKernelGGL((lsm_date_final_kernel<kLsmBlock, NB>), dim3(grid), dim3(kLsmBlock), 0, s, o, xs, vs, beta32,
                     wcash, tau, partials);
  return hipGetLastError();
}

hipError_t launch_lsm_dates(const DevOpt& o, const float* xs, const float* vs, const double* fac, float* wcash,
                            int32_t* tau, float* gpart, float* beta32, double* beta64, uint32_t* ticket,
                            double* partials, hipStream_t s, int nb) {
  if (nb == 10)
    return launch_lsm_dates_t<10>(o, xs, vs, fac, wcash, tau, gpart, beta32, beta64, ticket, partials, s);
  return hipErrorInvalidValue;
}

hipError_t launch_forward_ckpt(int scheme, const DevOpt& o, int ck, float* ckbuf, float* xN, double* partials,
                               hipStream_t s) {
  const int grid = (o.paths + kCkBlock - 1) / kCkBlock;
  if (scheme == 0)
    hipLaunchKernelGGL((forward_ckpt_kernel<kCkBlock, 0>), dim3(grid), dim3(kCkBlock), 0, s, o, ck, ckbuf, xN, partials);
  else if (scheme == 1)
    hipLaunchKernelGGL((forward_ckpt_kernel<kCkBlock, 1>), dim3(grid), dim3(kCkBlock), 0, s, o, ck, ckbuf, xN, partials);
  else if (scheme == 2)
    hipLaunchKernelGGL((forward_ckpt_kernel<kCkBlock, 2>), dim3(grid), dim3(kCkBlock), 0, s, o, ck, ckbuf, xN, partials);
  else if (scheme == 3)
    hipLaunchKernelGGL((forward_ckpt_kernel<kCkBlock, 3>), dim3(grid), dim3(kCkBlock), 0, s, o, ck, ckbuf, xN, partials);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

template <int B, int CK, bool EXT, int SCHEME>
static void adj_launch(const DevOpt& o, const float* ck_base, size_t ck_stride, const float* xstop,
                       const int32_t* tau, double* gpart, hipStream_t s) {
  const int grid = (o.paths + B - 1) / B;
  hipLaunchKernelGGL((adjoint_kernel<B, CK, EXT, SCHEME>), dim3(grid), dim3(B), 0, s, o, ck_base, ck_stride, xstop,
                     tau, gpart);
}

template <int SCHEME>
static hipError_t launch_adjoint_s(const DevOpt& o, int ck, int block, bool ext, const float* ck_base,
                                   size_t ck_stride, const float* xstop, const int32_t* tau, double* gpart,
                                   hipStream_t s) {
#define SIMR_ADJ(B, C, X)                                                        \
  if (block == B && ck == C && ext == X) {                                       \
    adj_launch<B, C, X, SCHEME>(o, ck_base, ck_stride, xstop, tau, gpart, s);    \
    return hipGetLastError();                                                    \
  }
  SIMR_ADJ(1024, 8, false) SIMR_ADJ(1024, 16, false) SIMR_ADJ(512, 8, false) SIMR_ADJ(512, 16, false)
  SIMR_ADJ(512, 32, false) SIMR_ADJ(256, 8, false) SIMR_ADJ(256, 16, false) SIMR_ADJ(256, 32, false)
  SIMR_ADJ(512, 8, true) SIMR_ADJ(512, 16, true) SIMR_ADJ(512, 32, true)
  SIMR_ADJ(256, 8, true) SIMR_ADJ(256, 16, true) SIMR_ADJ(256, 32, true)
#undef SIMR_ADJ
  return hipErrorInvalidValue;
}

hipError_t launch_adjoint(int scheme, const DevOpt& o, int ck, int block, bool ext, const float* ck_base,
                          size_t ck_stride, const float* xstop, const int32_t* tau, double* gpart, hipStream_t s) {
  if (scheme == 0) return launch_adjoint_s<0>(o, ck, block, ext, ck_base, ck_stride, xstop, tau, gpart, s);
  if (scheme == 1) return launch_adjoint_s<1>(o, ck, block, ext, ck_base, ck_stride, xstop, tau, gpart, s);
  if (scheme == 2) return launch_adjoint_s<2>(o, ck, block, ext, ck_base, ck_stride, xstop, tau, gpart, s);
  if (scheme == 3) return launch_adjoint_s<3>(o, ck, block, ext, ck_base, ck_stride, xstop, tau, gpart, s);
  return hipErrorInvalidValue;
}

hipError_t launch_debug_draws(uint64_t seed, uint32_t stream, int64_t path0, int64_t npaths, int32_t step0,
                              int32_t nsteps, uint32_t* words, float* unif, float* norm, hipStream_t s) {
  const int64_t total = npaths * nsteps;
  const int64_t grid = (total + 255) / 256;
  hipLaunchKernelGGL(debug_draws_kernel, dim3((uint32_t)grid), dim3(256), 0, s, (uint32_t)seed, (uint32_t)(seed >> 32),
                     stream, path0, npaths, step0, nsteps, words, unif, norm);
  return hipGetLastError();
}

hipError_t launch_debug_paths(int scheme, const DevOpt& o, float* xT, float* vT, float* pay, hipStream_t s) {
  const int grid = (o.paths + 255) / 256;
  if (scheme == 0) hipLaunchKernelGGL((debug_paths_kernel<0>), dim3(grid), dim3(256), 0, s, o, xT, vT, pay);
  else if (scheme == 1) hipLaunchKernelGGL((debug_paths_kernel<1>), dim3(grid), dim3(256), 0, s, o, xT, vT, pay);
  else if (scheme == 2) hipLaunchKernelGGL((debug_paths_kernel<2>), dim3(grid), dim3(256), 0, s, o, xT, vT, pay);
  else if (scheme == 3) hipLaunchKernelGGL((debug_paths_kernel<3>), dim3(grid), dim3(256), 0, s, o, xT, vT, pay);
  else if (scheme == 4) hipLaunchKernelGGL((debug_paths_kernel<4>), dim3(grid), dim3(256), 0, s, o, xT, vT, pay);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}


// ---------------------------------------------------------------------------------------------
// Correlated baskets.  One path per lane; a kernel instance serves every basket of d <= DMAX
// assets (the asset loops are unrolled to DMAX with wave-uniform guards i < d, so the
// correlation triangle and every per-asset state index are compile-time).  Asset i of
// transition n draws the Philox words of counter (n, path, stream, i); the asset normals are
// correlated, zc = L z2, and asset i takes its scheme's step with its own constants.
// ---------------------------------------------------------------------------------------------
namespace {

// Coefficient of the (correlated) asset normal in one log-price increment of the scheme.
template <int SCHEME>
__device__ __forceinline__ float z2_scale(const DevOpt& o, float v, float V) {
  if constexpr (SCHEME == 1)
    return o.sdt * fsqrt(fmaxf(v, 0.0f)) * o.srho;
  else
    return fsqrt(__builtin_fmaf(o.K3, v, o.K4 * V));
}

constexpr int tri(int i) { return i * (i + 1) / 2; }

// Forward tangents of the variance step in the two directions of the asset's own v0 (k = 0) and
// theta (k = 1): dv[k] the tangent of v, V the step's value (from the primal).  The primal's
// intermediate values are recomputed with the same operations.  QE: m and s^2 move with v and
// theta (dm = E dv + (1 - E) dtheta, ds^2 = A1 dv + dA2/dtheta dtheta), psi = s^2 / m^2, then the
// branch the step took; truncated Gaussian: mu / m and sigma / m in psi through the derivative
// table (0 above the table, where the last entry holds, and at V = 0).
template <int SCHEME>
__device__ __forceinline__ void variance_tan2(const DevOpt& o, float v, float V, float z1, float u,
                                              const float (&dv)[2], float (&dV)[2]) {
  const float m = __builtin_fmaf(v - o.theta, o.E, o.theta);
  const float s2 = __builtin_fmaf(v, o.A1, o.A2);
  float dm[2], ds2[2];
  dm[0] = dv[0] * o.E;
  dm[1] = __builtin_fmaf(dv[1], o.E, 1.0f - o.E);
  ds2[0] = dv[0] * o.A1;
  ds2[1] = __builtin_fmaf(dv[1], o.A1, o.dA2_dth);
  if (!(s2 > 0.0f)) {  // xi = 0: V = m
    dV[0] = dm[0];
    dV[1] = dm[1];
    return;
  }
  const float m2 = m * m;
  const float im2 = rcp(m2);
  const float psi = s2 * im2;
  float dpsi[2];
#pragma unroll
  for (int k = 0; k < 2; ++k) dpsi[k] = (ds2[k] - 2.0f * psi * m * dm[k]) * im2;
  if constexpr (SCHEME == 3) {
    const float lp = __builtin_amdgcn_logf(psi);  // log2
    float fm, fs, gpsi;  // g = fm + fs z1, gpsi = dg/dpsi
    if (lp < kTgLo) {
      fm = 1.0f;
      fs = fsqrt(psi);
      gpsi = z1 * 0.5f * rcp(fs);
    } else {
      const float traw = (lp - kTgLo) * kTgInvH;
      const bool flat = traw > (float)(kTgN - 1);
      const float t = fminf(traw, (float)(kTgN - 1));
      const int i = min((int)t, kTgN - 2);
      const float f = t - (float)i;
      const float2 a = o.tg[i], b = o.tg[i + 1];
      fm = __builtin_fmaf(f, b.x - a.x, a.x);
      fs = __builtin_amdgcn_exp2f(__builtin_fmaf(f, b.y - a.y, a.y));
      const float2 da = o.tg[kTgN + i], db = o.tg[kTgN + i + 1];
      const float dfm = __builtin_fmaf(f, db.x - da.x, da.x);
      const float dls = __builtin_fmaf(f, db.y - da.y, da.y);
      constexpr float kInvLn2 = 1.44269504088896340736f;
      const float ipsi = rcp(psi);
      gpsi = flat ? 0.0f : __builtin_fmaf(dfm * kInvLn2, ipsi, z1 * fs * dls * ipsi);
    }
    const float g = __builtin_fmaf(fs, z1, fm);
#pragma unroll
    for (int k = 0; k < 2; ++k) dV[k] = (m * g > 0.0f) ? __builtin_fmaf(dm[k], g, m * gpsi * dpsi[k]) : 0.0f;
  } else {
    if (psi <= kPsiC) {
      const float t = 2.0f * m2 * rcp(s2);  // 2 / psi
      const float q = fsqrt(t * (t - 1.0f));
      const float b2 = (t - 1.0f) + q;
      const float b = fsqrt(b2);
      const float ib = rcp(1.0f + b2);
      const float a = m * ib;
      const float bz = b + z1;
      const float db2_dt = 1.0f + (2.0f * t - 1.0f) * 0.5f * rcp(q);
      const float ipsi = rcp(psi);
#pragma unroll
      for (int k = 0; k < 2; ++k) {
        const float db2 = -t * dpsi[k] * ipsi * db2_dt;
        const float db = db2 * 0.5f * rcp(b);
        const float da = (dm[k] - a * db2) * ib;
        dV[k] = __builtin_fmaf(da, bz * bz, 2.0f * a * bz * db);
      }
    } else {
      const float pp1 = psi + 1.0f;
      const float p = (psi - 1.0f) * rcp(pp1);
      const float omp = 1.0f - p;
      const float iomp = rcp(omp);
      const float L = __builtin_amdgcn_logf(omp * rcp(1.0f - u)) * 0.69314718055994530942f;
#pragma unroll
      for (int k = 0; k < 2; ++k) {
        const float dp = 2.0f * dpsi[k] * rcp(pp1 * pp1);
        const float dL = -dp * iomp;
        // V = L m / (1 - p)
        dV[k] = (u <= p) ? 0.0f : __builtin_fmaf(__builtin_fmaf(dL, m, L * dm[k]), iomp, L * m * dp * iomp * iomp);
      }
    }
  }
  (void)V;
}

// One transition of an asset together with the forward tangents dx[k], dv[k] of its log-price
// and variance in its own v0 (k = 0) and theta (k = 1): the primal is transition<SCHEME> (the same
// operations, so the same path); QE and the truncated Gaussian step through QE's log-price step
// (C0 moves with theta), full-truncation Euler with the derivative of sqrt(v+) at 0 taken as 0.
// Returns the coefficient of the correlated normal d.z2 in the log-price increment.
template <int SCHEME>
__device__ __forceinline__ float transition_tan2(const DevOpt& o, float& x, float& v, float (&dx)[2], float (&dv)[2],
                                                 const Draw& d) {
  static_assert(SCHEME == 0 || SCHEME == 1 || SCHEME == 3, "tangents for QE, full-truncation Euler and TG");
  const float vb = v;
  if constexpr (SCHEME == 1) {
    const float vp = fmaxf(vb, 0.0f);
    const float sv = fsqrt(vp);
    fte_step(o, x, v, d.z1, d.z2);
    const float zs = __builtin_fmaf(o.rho, d.z1, o.srho * d.z2);
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      const float dvp = vb > 0.0f ? dv[k] : 0.0f;
      const float dsv = sv > 0.0f ? dvp * 0.5f * rcp(sv) : 0.0f;
      dx[k] = __builtin_fmaf(o.sdt * dsv, zs, __builtin_fmaf(-o.hdt, dvp, dx[k]));
      const float dth = k == 1 ? o.kdt : 0.0f;  // d(kappa theta dt)/dtheta
      dv[k] = __builtin_fmaf(o.xisdt * dsv, d.z1, __builtin_fmaf(-o.kdt, dvp, dv[k] + dth));
    }
    return o.sdt * sv * o.srho;
  } else {
    const float V = SCHEME == 3 ? tg_variance(o, vb, d.z1) : qe_variance(o, vb, d.z1, d.u);
    float dV[2];
    variance_tan2<SCHEME>(o, vb, V, d.z1, d.u, dv, dV);
    const float w = __builtin_fmaf(o.K3, vb, o.K4 * V);
    const float sw = fsqrt(w);
    x += qe_logprice_inc(o, vb, V, d.z2);
    const float hw = w > 0.0f ? 0.5f * rcp(sw) * d.z2 : 0.0f;
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      float t = __builtin_fmaf(o.K2, dV[k], __builtin_fmaf(o.K1, dv[k], k == 1 ? o.dC0_dth : 0.0f));
      t = __builtin_fmaf(__builtin_fmaf(o.K3, dv[k], o.K4 * dV[k]), hw, t);
      dx[k] += t;
      dv[k] = dV[k];
    }
    v = V;
    return sw;
  }
}

}  // namespace

// MODE 0: price -- block sums {sum X, sum X^2} of X = e^{-rT} h(B_T) into rows[2 block + c];
//         o1/o2 (may be null): ln(S_T,i / S0_i) and v_T,i at [p d + i], o3: X per path.
// MODE 1: Greeks records, column-major (column c at o1[c P]): c = 0 the discounted cash flow,
//         1 + i the pathwise delta sample D_i, 1 + d + j the likelihood-ratio score W_j of
//         ln S0_j (sum_n s_nj u_nj / sum_n s_nj^2, u_n = L^{-T} z2_n).  With tau (per-path
//         stopping index), the paths stop there and the scores are not formed (0).
// MODE 2: Longstaff-Schwartz write-out: o1[(n - 1) P + p] = ln(B_n / B_0),
//         o2[...] = sum_i w_i S_i,n max(v_i,n, 0) / B_n; first zeroes zero[0, nzero).
// MODE 3: risk records (QE, full-truncation Euler, truncated Gaussian; DMAX <= 8), column-major:
//         c = 0 the discounted (stopped) cash flow X, 1 + i the vega sample dX/dv0_i, 1 + d + i
//         dX/dtheta_i, 1 + 2 d + q the correlation sample dX/dC_ij of pair q = i (i - 1) / 2 + j
//         (i > j): with a_k = e^{-r tau dt} h'(B) w_k S_k and Q_km = sum_n s_nk z2_nm (m <= k),
//         sum_k a_k sum_m dl[q kRiskTri + tri(k) + m] Q_km, dl the derivative of the Cholesky
//         factor when C_ij and C_ji move together.  With tau the paths stop there.
template <int SCHEME, int DMAX, int MODE>
__global__ __launch_bounds__(256) void basket_path_kernel(const DevBasket* __restrict__ bk,
                                                          const DevOpt* __restrict__ ao,
                                                          const int32_t* __restrict__ tau, float* __restrict__ o1,
                                                          float* __restrict__ o2, float* __restrict__ o3,
                                                          uint32_t* __restrict__ zero, int64_t nzero,
                                                          double* __restrict__ rows, const float* __restrict__ dl) {
  const DevBasket& B = *bk;
  const uint32_t p = blockIdx.x * 256 + threadIdx.x;
  if constexpr (MODE == 2) {
    for (int64_t i = p; i < nzero; i += (int64_t)gridDim.x * 256) zero[i] = 0u;
  }
  const int d = B.d;
  const size_t P = (size_t)B.paths;
  const bool live = p < (uint32_t)B.paths;
  float x[DMAX], v[DMAX], sa[DMAX], sb[DMAX];
#pragma unroll
  for (int i = 0; i < DMAX; ++i) {
    x[i] = 0.0f;
    v[i] = i < d ? ao[i].v0 : 0.0f;
    sa[i] = 0.0f;
    sb[i] = 0.0f;
  }
  int32_t nstop = live ? B.steps : 0;
  if constexpr (MODE == 1 || MODE == 3) {
    if (tau && live) nstop = tau[p];
  }
  static_assert(MODE != 3 || DMAX <= kRiskMaxAssets, "risk records for at most 8 assets");
  constexpr int NT = MODE == 3 ? DMAX : 1;  // the risk mode's tangents and Q sums
  float tx[NT][2], tv[NT][2], Q[tri(NT)];
  if constexpr (MODE == 3) {
#pragma unroll
    for (int i = 0; i < NT; ++i) {
      tx[i][0] = tx[i][1] = 0.0f;
      tv[i][0] = 1.0f;  // dv0/dv0
      tv[i][1] = 0.0f;
    }
#pragma unroll
    for (int q = 0; q < tri(NT); ++q) Q[q] = 0.0f;
  }
  for (int32_t n = 0; n < nstop; ++n) {
    float z2[DMAX], s[DMAX];
#pragma unroll
    for (int i = 0; i < DMAX; ++i) {
      z2[i] = 0.0f;
      s[i] = 0.0f;
      if (i < d) {
        const Words w = philox4x32_10((uint32_t)n, p, B.stream, (uint32_t)i, B.seed_lo, B.seed_hi);
        Draw dr;
        box_muller(u01(w.w0), u01(w.w1), dr.z1, z2[i]);
        dr.u = u01(w.w2);
        float zc = 0.0f;
#pragma unroll
        for (int k = 0; k <= i; ++k) zc = __builtin_fmaf(B.L[tri(i) + k], z2[k], zc);
        dr.z2 = zc;
        const float vb = v[i];
        if constexpr (MODE == 3) {
          s[i] = transition_tan2<SCHEME>(ao[i], x[i], v[i], tx[i < NT ? i : 0], tv[i < NT ? i : 0], dr);
        } else {
          transition<SCHEME>(ao[i], x[i], v[i], dr);
          if constexpr (MODE == 1) s[i] = z2_scale<SCHEME>(ao[i], vb, v[i]);
        }
      }
    }
    if constexpr (MODE == 3) {
#pragma unroll
      for (int k = 0; k < NT; ++k)
#pragma unroll
        for (int m = 0; m <= k; ++m) Q[tri(k) + m] = __builtin_fmaf(s[k], z2[m], Q[tri(k) + m]);
    }
    if constexpr (MODE == 1) {
      if (tau == nullptr) {
#pragma unroll
        for (int j = 0; j < DMAX; ++j) {
          if (j < d) {
            float uj = 0.0f;  // (L^{-T} z2)_j = sum_{k >= j} (L^{-1})_kj z2_k
#pragma unroll
            for (int k = j; k < DMAX; ++k)
              if (k < d) uj = __builtin_fmaf(B.Linv[tri(k) + j], z2[k], uj);
            sa[j] = __builtin_fmaf(s[j], uj, sa[j]);
            sb[j] = __builtin_fmaf(s[j], s[j], sb[j]);
          }
        }
      }
    }
    if constexpr (MODE == 2) {
      float Bn = 0.0f, Bv = 0.0f;
#pragma unroll
      for (int i = 0; i < DMAX; ++i) {
        if (i < d) {
          const float Si = B.wS0[i] * __builtin_amdgcn_exp2f(x[i] * 1.44269504088896340736f);
          Bn += Si;
          Bv = __builtin_fmaf(Si, fmaxf(v[i], 0.0f), Bv);
        }
      }
      o1[(size_t)n * P + p] = __builtin_amdgcn_logf(Bn * B.invB0) * 0.69314718055994530942f;
      o2[(size_t)n * P + p] = Bv * rcp(Bn);
    }
  }
  if constexpr (MODE == 0 || MODE == 1 || MODE == 3) {
    float e[DMAX];
    float Bt = 0.0f;
#pragma unroll
    for (int i = 0; i < DMAX; ++i) {
      e[i] = 0.0f;
      if (i < d) {
        e[i] = __builtin_amdgcn_exp2f(x[i] * 1.44269504088896340736f);
        Bt += B.wS0[i] * e[i];
      }
    }
    const bool call = B.payoff == 0 || B.payoff == 3;
    const float h = fmaxf(call ? Bt - B.K : B.K - Bt, 0.0f);
    if constexpr (MODE == 0) {
      const float X = live ? B.disc * h : 0.0f;
      if (live) {
#pragma unroll
        for (int i = 0; i < DMAX; ++i) {
          if (i < d) {
            if (o1) o1[(size_t)p * d + i] = x[i];
            if (o2) o2[(size_t)p * d + i] = v[i];
          }
        }
        if (o3) o3[p] = X;
      }
      __shared__ double s_red[2 * (256 / kWave)];
      double vals[2] = {(double)X, (double)X * (double)X};
      block_sum<256, 2, double>(vals, s_red);
      if (threadIdx.x == 0) {
        rows[2 * (size_t)blockIdx.x] = vals[0];
        rows[2 * (size_t)blockIdx.x + 1] = vals[1];
      }
    } else if (live && MODE == 1) {
      const float dsc = __builtin_amdgcn_exp2f(-B.rdt * 1.44269504088896340736f * (float)nstop);
      const float dh = h > 0.0f ? (call ? dsc : -dsc) : 0.0f;
      o1[p] = dsc * h;
#pragma unroll
      for (int i = 0; i < DMAX; ++i) {
        if (i < d) {
          o1[(size_t)(1 + i) * P + p] = dh * B.w[i] * e[i];
          o1[(size_t)(1 + d + i) * P + p] = tau ? 0.0f : sa[i] / sb[i];  // 0 / 0 = NaN: no score
        }
      }
    } else if (live) {  // MODE 3
      const float dsc = __builtin_amdgcn_exp2f(-B.rdt * 1.44269504088896340736f * (float)nstop);
      const float dh = h > 0.0f ? (call ? dsc : -dsc) : 0.0f;
      o1[p] = dsc * h;
      float a[NT];
#pragma unroll
      for (int i = 0; i < NT; ++i) {
        a[i] = i < d ? dh * B.wS0[i] * e[i] : 0.0f;
        if (i < d) {
          o1[(size_t)(1 + i) * P + p] = a[i] * tx[i][0];
          o1[(size_t)(1 + d + i) * P + p] = a[i] * tx[i][1];
        }
      }
#pragma unroll
      for (int i = 1; i < NT; ++i) {
#pragma unroll
        for (int j = 0; j < i; ++j) {
          if (i < d) {
            const int q = tri(i - 1) + j;
            const float* dq = dl + (size_t)q * kRiskTri;
            float g = 0.0f;
#pragma unroll
            for (int k = i; k < NT; ++k) {  // the rows of dL above i are 0 for this pair
              float t = 0.0f;
#pragma unroll
              for (int m = 0; m <= k; ++m) t = __builtin_fmaf(dq[tri(k) + m], Q[tri(k) + m], t);
              g = __builtin_fmaf(a[k], t, g);
            }
            o1[(size_t)(1 + 2 * d + q) * P + p] = g;
          }
        }
      }
    }
  }
}

// Few paths, many assets: LPP consecutive lanes of a wave per path, lane s of a path owning the
// assets [s A, s A + A), A = DMAX / LPP, so that small path counts still fill the chip.  The
// per-asset constants, L and L^{-1} are copied to LDS (the asset indices differ between lanes);
// the independent asset normals of a step pass through LDS; the basket sums are folded across
// the path's lanes by shuffles.  Every lane runs all N steps (dead lanes and, in MODE 1, paths
// past their stopping index draw but do not step), so the two block barriers per step are
// uniform.  Modes and outputs as basket_path_kernel (the FP32 basket sums are added in another
// order, a rounding-level difference).
template <int SCHEME, int DMAX, int LPP, int MODE>
__global__ __launch_bounds__(256) void basket_split_kernel(const DevBasket* __restrict__ bk,
                                                           const DevOpt* __restrict__ ao,
                                                           const int32_t* __restrict__ tau, float* __restrict__ o1,
                                                           float* __restrict__ o2, float* __restrict__ o3,
                                                           uint32_t* __restrict__ zero, int64_t nzero,
                                                           double* __restrict__ rows) {
  constexpr int A = DMAX / LPP;
  constexpr int PB = 256 / LPP;  // paths per block
  static_assert(kWave % LPP == 0 && DMAX % LPP == 0, "a path's lanes lie in one wave");
  __shared__ DevOpt s_ao[DMAX];
  __shared__ float s_L[DMAX * (DMAX + 1) / 2];
  __shared__ float s_Li[MODE == 1 ? DMAX * (DMAX + 1) / 2 : 1];
  __shared__ float s_z[PB * (DMAX + 1)];
  const DevBasket& B = *bk;
  const int d = B.d;
  const int t = threadIdx.x;
  if constexpr (MODE == 2) {
    for (int64_t i = (int64_t)blockIdx.x * 256 + t; i < nzero; i += (int64_t)gridDim.x * 256) zero[i] = 0u;
  }
  {
    const uint32_t* src = (const uint32_t*)ao;
    uint32_t* dst = (uint32_t*)s_ao;
    const int nw = d * (int)(sizeof(DevOpt) / 4);
    for (int w = t; w < nw; w += 256) dst[w] = src[w];
    const int nt = d * (d + 1) / 2;
    for (int w = t; w < nt; w += 256) {
      s_L[w] = B.L[w];
      if constexpr (MODE == 1) s_Li[w] = B.Linv[w];
    }
  }
  __syncthreads();
  const int pl = t / LPP, sub = t % LPP;
  const uint32_t p = blockIdx.x * PB + pl;
  const size_t P = (size_t)B.paths;
  const bool live = p < (uint32_t)B.paths;
  const int i0 = sub * A;
  float x[A], v[A], sa[A], sb[A];
#pragma unroll
  for (int j = 0; j < A; ++j) {
    x[j] = 0.0f;
    v[j] = i0 + j < d ? s_ao[i0 + j].v0 : 0.0f;
    sa[j] = 0.0f;
    sb[j] = 0.0f;
  }
  int32_t nstop = live ? B.steps : 0;
  if constexpr (MODE == 1) {
    if (tau && live) nstop = tau[p];
  }
  float* zrow = s_z + pl * (DMAX + 1);
  for (int32_t n = 0; n < B.steps; ++n) {
    float z1[A], u[A];
#pragma unroll
    for (int j = 0; j < A; ++j) {
      const int i = i0 + j;
      z1[j] = 0.0f;
      u[j] = 0.5f;
      if (i < d) {
        const Words w = philox4x32_10((uint32_t)n, p, B.stream, (uint32_t)i, B.seed_lo, B.seed_hi);
        float z2;
        box_muller(u01(w.w0), u01(w.w1), z1[j], z2);
        u[j] = u01(w.w2);
        zrow[i] = z2;
      }
    }
    __syncthreads();
    const bool step = n < nstop;
    float s[A];
#pragma unroll
    for (int j = 0; j < A; ++j) {
      const int i = i0 + j;
      s[j] = 0.0f;
      if (i < d && step) {
        float zc = 0.0f;
        const float* Lrow = s_L + i * (i + 1) / 2;
        for (int k = 0; k <= i; ++k) zc = __builtin_fmaf(Lrow[k], zrow[k], zc);
        Draw dr;
        dr.z1 = z1[j];
        dr.z2 = zc;
        dr.u = u[j];
        dr.u2 = 0.5f;
        const float vb = v[j];
        transition<SCHEME>(s_ao[i], x[j], v[j], dr);
        if constexpr (MODE == 1) s[j] = z2_scale<SCHEME>(s_ao[i], vb, v[j]);
      }
    }
    if constexpr (MODE == 1) {
      if (tau == nullptr && step) {
#pragma unroll
        for (int j = 0; j < A; ++j) {
          const int i = i0 + j;
          if (i < d) {
            float uj = 0.0f;  // (L^{-T} z2)_i = sum_{k >= i} (L^{-1})_ki z2_k
            for (int k = i; k < d; ++k) uj = __builtin_fmaf(s_Li[k * (k + 1) / 2 + i], zrow[k], uj);
            sa[j] = __builtin_fmaf(s[j], uj, sa[j]);
            sb[j] = __builtin_fmaf(s[j], s[j], sb[j]);
          }
        }
      }
    }
    if constexpr (MODE == 2) {
      float Bn = 0.0f, Bv = 0.0f;
#pragma unroll
      for (int j = 0; j < A; ++j) {
        const int i = i0 + j;
        if (i < d) {
          const float Si = B.wS0[i] * __builtin_amdgcn_exp2f(x[j] * 1.44269504088896340736f);
          Bn += Si;
          Bv = __builtin_fmaf(Si, fmaxf(v[j], 0.0f), Bv);
        }
      }
#pragma unroll
      for (int off = 1; off < LPP; off <<= 1) {
        Bn += __shfl_xor(Bn, off, kWave);
        Bv += __shfl_xor(Bv, off, kWave);
      }
      if (sub == 0 && live) {
        o1[(size_t)n * P + p] = __builtin_amdgcn_logf(Bn * B.invB0) * 0.69314718055994530942f;
        o2[(size_t)n * P + p] = Bv * rcp(Bn);
      }
    }
    __syncthreads();  // the step's normals are overwritten by the next
  }
  if constexpr (MODE == 0 || MODE == 1) {
    float e[A];
    float Bt = 0.0f;
#pragma unroll
    for (int j = 0; j < A; ++j) {
      e[j] = 0.0f;
      if (i0 + j < d) {
        e[j] = __builtin_amdgcn_exp2f(x[j] * 1.44269504088896340736f);
        Bt += B.wS0[i0 + j] * e[j];
      }
    }
#pragma unroll
    for (int off = 1; off < LPP; off <<= 1) Bt += __shfl_xor(Bt, off, kWave);
    const bool call = B.payoff == 0 || B.payoff == 3;
    const float h = fmaxf(call ? Bt - B.K : B.K - Bt, 0.0f);
    if constexpr (MODE == 0) {
      const float X = (live && sub == 0) ? B.disc * h : 0.0f;
      if (live) {
#pragma unroll
        for (int j = 0; j < A; ++j) {
          if (i0 + j < d) {
            if (o1) o1[(size_t)p * d + i0 + j] = x[j];
            if (o2) o2[(size_t)p * d + i0 + j] = v[j];
          }
        }
        if (o3 && sub == 0) o3[p] = X;
      }
      __shared__ double s_red[2 * (256 / kWave)];
      double vals[2] = {(double)X, (double)X * (double)X};
      block_sum<256, 2, double>(vals, s_red);
      if (threadIdx.x == 0) {
        rows[2 * (size_t)blockIdx.x] = vals[0];
        rows[2 * (size_t)blockIdx.x + 1] = vals[1];
      }
    } else if (live) {
      const float dsc = __builtin_amdgcn_exp2f(-B.rdt * 1.44269504088896340736f * (float)nstop);
      const float dh = h > 0.0f ? (call ? dsc : -dsc) : 0.0f;
      if (sub == 0) o1[p] = dsc * h;
#pragma unroll
      for (int j = 0; j < A; ++j) {
        const int i = i0 + j;
        if (i < d) {
          o1[(size_t)(1 + i) * P + p] = dh * B.w[i] * e[j];
          o1[(size_t)(1 + d + i) * P + p] = tau ? 0.0f : sa[j] / sb[j];  // 0 / 0 = NaN: no score
        }
      }
    }
  }
}

// Moments of the Greeks records over one chunk of kBasketChunk paths (one block), in FP64 and
// path order: column q = 0, 1: X, X^2; 2 + i, 2 + d + i: D_i, D_i^2; then for every pair
// i <= j in row order, g_ij and g_ij^2 with the symmetrised pathwise-likelihood-ratio sample
// g_ij = (D_i W_j / S0_j + D_j W_i / S0_i) / 2 - [i = j] D_i / S0_i (0 on a path whose D are
// all 0).  part[chunk ncol + q].
__global__ __launch_bounds__(256) void basket_moments_kernel(const DevBasket* __restrict__ bk,
                                                             const float* __restrict__ rec, int32_t ncol,
                                                             double* __restrict__ part) {
  __shared__ float s_rec[(1 + 2 * kMaxAssets) * (kBasketChunk + 1)];  // padded rows: no bank conflicts
  __shared__ int32_t s_any[kBasketChunk];
  const DevBasket& B = *bk;
  const int d = B.d;
  const int R = 1 + 2 * d;
  const int64_t P = B.paths;
  const int64_t p0 = (int64_t)blockIdx.x * kBasketChunk;
  const int np = (int)min((int64_t)kBasketChunk, P - p0);
  for (int idx = threadIdx.x; idx < R * kBasketChunk; idx += 256) {
    const int c = idx / kBasketChunk, t = idx % kBasketChunk;
    s_rec[c * (kBasketChunk + 1) + t] = t < np ? rec[(size_t)c * P + p0 + t] : 0.0f;
  }
  __syncthreads();
  for (int t = threadIdx.x; t < kBasketChunk; t += 256) {
    int any = 0;
    for (int i = 0; i < d; ++i) any |= s_rec[(1 + i) * (kBasketChunk + 1) + t] != 0.0f;
    s_any[t] = any;
  }
  __syncthreads();
  for (int q = threadIdx.x; q < ncol; q += 256) {
    double acc = 0.0;
    if (q < 2 + 2 * d) {
      const int c = q < 2 ? 0 : (q < 2 + d ? q - 1 : q - 1 - d);
      const bool sq = q == 1 || q >= 2 + d;
      const float* col = s_rec + c * (kBasketChunk + 1);
      for (int t = 0; t < np; ++t) {
        const double xv = (double)col[t];
        acc += sq ? xv * xv : xv;
      }
    } else {
      const int pr = (q - 2 - 2 * d) >> 1;
      const bool sq = ((q - 2 - 2 * d) & 1) != 0;
      int i = 0, rem = pr;
      while (rem >= d - i) {
        rem -= d - i;
        ++i;
      }
      const int j = i + rem;
      const double iSi = 1.0 / (double)B.S0[i], iSj = 1.0 / (double)B.S0[j];
      const float* Di = s_rec + (1 + i) * (kBasketChunk + 1);
      const float* Dj = s_rec + (1 + j) * (kBasketChunk + 1);
      const float* Wi = s_rec + (1 + d + i) * (kBasketChunk + 1);
      const float* Wj = s_rec + (1 + d + j) * (kBasketChunk + 1);
      for (int t = 0; t < np; ++t) {
        double g = 0.0;
        if (s_any[t]) {
          g = 0.5 * ((double)Di[t] * (double)Wj[t] * iSj + (double)Dj[t] * (double)Wi[t] * iSi);
          if (i == j) g -= (double)Di[t] * iSi;
        }
        acc += sq ? g * g : g;
      }
    }
    part[(size_t)blockIdx.x * ncol + q] = acc;
  }
}

int basket_tier(int d) { return d <= 4 ? 4 : d <= 8 ? 8 : d <= 16 ? 16 : 32; }

int basket_lanes_per_path(int d, int64_t paths, int num_cus) {
  // one lane per path with at least 2 waves per SIMD already, or too few assets to share (5 assets
  // over 2 lanes ran slower than one lane per path on the 25,000-path Table 1 basket); else the
  // fewest lanes per path (4, 8, 16, and 32 for more than 16 assets) that reach 6 waves per SIMD,
  // or the most.  On the 25,000-path Table 1 baskets of 10 / 20 / 30 assets, 4 / 8 / 16 lanes
  // took 1.00 / 0.89 / 0.82, 2.86 / 2.47 / 2.18 and 6.19 / 5.34 / 4.76 ms (32 lanes no faster);
  // the Greeks of 32 assets on 6,000 paths 1.66 / 1.12 / 0.81 / 0.65 ms at 4 / 8 / 16 / 32: the
  // step's transcendental and Philox chains need the extra waves to hide their latency.
  if (d <= 8 || (paths + kWave - 1) / kWave >= 2 * 4 * (int64_t)num_cus) return 1;
  const int64_t target = 6 * 4 * (int64_t)num_cus;
  const int most = d > 16 ? 32 : 16;
  for (int l = 4; l < most; l *= 2)
    if ((paths * l + kWave - 1) / kWave >= target) return l;
  return most;
}

template <int SCHEME, int DMAX, int LPP>
static hipError_t launch_split_t(int mode, int64_t paths, const DevBasket* bk, const DevOpt* ao, const int32_t* tau,
                                 float* o1, float* o2, float* o3, uint32_t* zero, int64_t nzero, double* rows,
                                 hipStream_t s) {
  constexpr int PB = 256 / LPP;
  const int grid = (int)((paths + PB - 1) / PB);
  if (mode == 0)
    hipLaunchKernelGGL((basket_split_kernel<SCHEME, DMAX, LPP, 0>), dim3(grid), dim3(256), 0, s, bk, ao, tau, o1, o2,
                       o3, zero, nzero, rows);
  else if (mode == 1)
    hipLaunchKernelGGL((basket_split_kernel<SCHEME, DMAX, LPP, 1>), dim3(grid), dim3(256), 0, s, bk, ao, tau, o1, o2,
                       o3, zero, nzero, rows);
  else
    hipLaunchKernelGGL((basket_split_kernel<SCHEME, DMAX, LPP, 2>), dim3(grid), dim3(256), 0, s, bk, ao, tau, o1, o2,
                       o3, zero, nzero, rows);
  return hipGetLastError();
}

template <int SCHEME>
static hipError_t launch_split_s(int mode, int d, int lpp, int64_t paths, const DevBasket* bk, const DevOpt* ao,
                                 const int32_t* tau, float* o1, float* o2, float* o3, uint32_t* zero, int64_t nzero,
                                 double* rows, hipStream_t s) {
  if (d <= 16) {
    if (lpp > 16) return hipErrorInvalidValue;
    if (lpp == 4) return launch_split_t<SCHEME, 16, 4>(mode, paths, bk, ao, tau, o1, o2, o3, zero, nzero, rows, s);
    if (lpp == 8) return launch_split_t<SCHEME, 16, 8>(mode, paths, bk, ao, tau, o1, o2, o3, zero, nzero, rows, s);
    return launch_split_t<SCHEME, 16, 16>(mode, paths, bk, ao, tau, o1, o2, o3, zero, nzero, rows, s);
  }
  if (lpp == 4) return launch_split_t<SCHEME, 32, 4>(mode, paths, bk, ao, tau, o1, o2, o3, zero, nzero, rows, s);
  if (lpp == 8) return launch_split_t<SCHEME, 32, 8>(mode, paths, bk, ao, tau, o1, o2, o3, zero, nzero, rows, s);
  if (lpp == 16) return launch_split_t<SCHEME, 32, 16>(mode, paths, bk, ao, tau, o1, o2, o3, zero, nzero, rows, s);
  return launch_split_t<SCHEME, 32, 32>(mode, paths, bk, ao, tau, o1, o2, o3, zero, nzero, rows, s);
}

template <int SCHEME, int DMAX>
static hipError_t launch_basket_t(int mode, int grid, const DevBasket* bk, const DevOpt* ao, const int32_t* tau,
                                  float* o1, float* o2, float* o3, uint32_t* zero, int64_t nzero, double* rows,
                                  hipStream_t s) {
  const float* nodl = nullptr;
  if (mode == 0)
    hipLaunchKernelGGL((basket_path_kernel<SCHEME, DMAX, 0>), dim3(grid), dim3(256), 0, s, bk, ao, tau, o1, o2, o3,
                       zero, nzero, rows, nodl);
  else if (mode == 1)
    hipLaunchKernelGGL((basket_path_kernel<SCHEME, DMAX, 1>), dim3(grid), dim3(256), 0, s, bk, ao, tau, o1, o2, o3,
                       zero, nzero, rows, nodl);
  else
    hipLaunchKernelGGL((basket_path_kernel<SCHEME, DMAX, 2>), dim3(grid), dim3(256), 0, s, bk, ao, tau, o1, o2, o3,
                       zero, nzero, rows, nodl);
  return hipGetLastError();
}

template <int SCHEME, int DMAX>
static hipError_t launch_risk_t(int grid, const DevBasket* bk, const DevOpt* ao, const int32_t* tau, float* rec,
                                const float* dl, hipStream_t s) {
  hipLaunchKernelGGL((basket_path_kernel<SCHEME, DMAX, 3>), dim3(grid), dim3(256), 0, s, bk, ao, tau, rec,
                     (float*)nullptr, (float*)nullptr, (uint32_t*)nullptr, (int64_t)0, (double*)nullptr, dl);
  return hipGetLastError();
}

template <int SCHEME>
static hipError_t launch_risk_s(int d, int grid, const DevBasket* bk, const DevOpt* ao, const int32_t* tau, float* rec,
                                const float* dl, hipStream_t s) {
  return d <= 4 ? launch_risk_t<SCHEME, 4>(grid, bk, ao, tau, rec, dl, s)
                : launch_risk_t<SCHEME, 8>(grid, bk, ao, tau, rec, dl, s);
}

hipError_t launch_basket_risk(int scheme, int d, int64_t paths, const DevBasket* bk, const DevOpt* ao,
                              const int32_t* tau, float* rec, const float* dl, hipStream_t s) {
  if (d < 1 || d > kRiskMaxAssets) return hipErrorInvalidValue;
  const int grid = (int)((paths + 255) / 256);
  switch (scheme) {
    case 0: return launch_risk_s<0>(d, grid, bk, ao, tau, rec, dl, s);
    case 1: return launch_risk_s<1>(d, grid, bk, ao, tau, rec, dl, s);
    case 3: return launch_risk_s<3>(d, grid, bk, ao, tau, rec, dl, s);
    default: return hipErrorInvalidValue;
  }
}

// Per chunk of kBasketChunk paths, the FP64 sums of every record column and of its square, in
// path order: part[chunk * 2 ncol + 2 c] = sum x, [.. + 1] = sum x^2 (column c at rec[c P]).
// The columns of a chunk are staged through LDS (coalesced loads along the paths).
__global__ __launch_bounds__(256) void record_moments_kernel(const float* __restrict__ rec, int32_t ncol, int64_t P,
                                                             double* __restrict__ part) {
  __shared__ float s_rec[kRiskRecCols * (kBasketChunk + 1)];  // padded rows: no bank conflicts
  const int64_t p0 = (int64_t)blockIdx.x * kBasketChunk;
  const int np = (int)min((int64_t)kBasketChunk, P - p0);
  for (int idx = threadIdx.x; idx < ncol * kBasketChunk; idx += 256) {
    const int c = idx / kBasketChunk, t = idx % kBasketChunk;
    s_rec[c * (kBasketChunk + 1) + t] = t < np ? rec[(size_t)c * P + p0 + t] : 0.0f;
  }
  __syncthreads();
  for (int q = threadIdx.x; q < 2 * ncol; q += 256) {
    const float* col = s_rec + (q >> 1) * (kBasketChunk + 1);
    double acc = 0.0;
    if (q & 1) {
      for (int t = 0; t < np; ++t) acc += (double)col[t] * (double)col[t];
    } else {
      for (int t = 0; t < np; ++t) acc += (double)col[t];
    }
    part[(size_t)blockIdx.x * 2 * ncol + q] = acc;
  }
}

hipError_t launch_record_moments(const float* rec, int ncol, int64_t paths, double* part, hipStream_t s) {
  if (ncol < 1 || ncol > kRiskRecCols) return hipErrorInvalidValue;
  const int grid = (int)((paths + kBasketChunk - 1) / kBasketChunk);
  hipLaunchKernelGGL(record_moments_kernel, dim3(grid), dim3(256), 0, s, rec, ncol, paths, part);
  return hipGetLastError();
}

template <int SCHEME>
static hipError_t launch_basket_s(int mode, int d, int grid, const DevBasket* bk, const DevOpt* ao,
                                  const int32_t* tau, float* o1, float* o2, float* o3, uint32_t* zero, int64_t nzero,
                                  double* rows, hipStream_t s) {
  switch (basket_tier(d)) {
    case 4: return launch_basket_t<SCHEME, 4>(mode, grid, bk, ao, tau, o1, o2, o3, zero, nzero, rows, s);
    case 8: return launch_basket_t<SCHEME, 8>(mode, grid, bk, ao, tau, o1, o2, o3, zero, nzero, rows, s);
    case 16: return launch_basket_t<SCHEME, 16>(mode, grid, bk, ao, tau, o1, o2, o3, zero, nzero, rows, s);
    default: return launch_basket_t<SCHEME, 32>(mode, grid, bk, ao, tau, o1, o2, o3, zero, nzero, rows, s);
  }
}

hipError_t launch_basket_paths(int scheme, int mode, int d, int64_t paths, int lpp, const DevBasket* bk,
                               const DevOpt* ao, const int32_t* tau, float* o1, float* o2, float* o3, uint32_t* zero,
                               int64_t nzero, double* rows, hipStream_t s) {
  if (d < 1 || d > kMaxAssets || mode < 0 || mode > 2) return hipErrorInvalidValue;
  if (lpp > 1) {
    if (d <= 8 || (lpp != 4 && lpp != 8 && lpp != 16 && lpp != 32)) return hipErrorInvalidValue;
    switch (scheme) {
      case 0: return launch_split_s<0>(mode, d, lpp, paths, bk, ao, tau, o1, o2, o3, zero, nzero, rows, s);
      case 1: return launch_split_s<1>(mode, d, lpp, paths, bk, ao, tau, o1, o2, o3, zero, nzero, rows, s);
      case 2: return launch_split_s<2>(mode, d, lpp, paths, bk, ao, tau, o1, o2, o3, zero, nzero, rows, s);
      case 3: return launch_split_s<3>(mode, d, lpp, paths, bk, ao, tau, o1, o2, o3, zero, nzero, rows, s);
      default: return hipErrorInvalidValue;
    }
  }
  const int grid = (int)((paths + 255) / 256);
  switch (scheme) {
    case 0: return launch_basket_s<0>(mode, d, grid, bk, ao, tau, o1, o2, o3, zero, nzero, rows, s);
    case 1: return launch_basket_s<1>(mode, d, grid, bk, ao, tau, o1, o2, o3, zero, nzero, rows, s);
    case 2: return launch_basket_s<2>(mode, d, grid, bk, ao, tau, o1, o2, o3, zero, nzero, rows, s);
    case 3: return launch_basket_s<3>(mode, d, grid, bk, ao, tau, o1, o2, o3, zero, nzero, rows, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_basket_moments(const DevBasket* bk, int64_t paths, const float* rec, int ncol, double* part,
                                 hipStream_t s) {
  const int grid = (int)((paths + kBasketChunk - 1) / kBasketChunk);
  hipLaunchKernelGGL(basket_moments_kernel, dim3(grid), dim3(256), 0, s, bk, rec, ncol, part);
  return hipGetLastError();
}

}  // namespace simr
