// valu_issue_probe.hip -- issue rate of single VALU instruction kinds on gfx950, the measured
// basis of the instruction-issue view of the VALU-bound kernels (a transcendental issues at half
// the rate of a plain FP32 instruction; some integer bit operations co-issue beside an FMA).
//
// Every lane of a grid of 8 blocks of 256 threads per CU runs ITER iterations of CH independent
// dependency chains of one instruction kind (or, for the pairs, half the chains of each kind).
// Each thread writes one word, so nothing is dead code; the output buffer holds one word per
// thread.  Prints one JSON line: wave instructions per second of the whole chip for each kind
// (best of three timed launches after one untimed launch).
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <vector>

constexpr int CH = 8;
constexpr int ITER = 4096;

#define SINGLE(NAME, T, INIT, BODY)                                                        \
  __global__ __launch_bounds__(256) void NAME(T seed, T k, uint32_t* out, int n) {         \
    const int t = blockIdx.x * 256 + threadIdx.x;                                            \
    T a[CH];                                                                                 \
    _Pragma("unroll") for (int j = 0; j < CH; ++j) a[j] = INIT;                             \
    for (int it = 0; it < ITER; ++it) {                                                      \
      _Pragma("unroll") for (int j = 0; j < CH; ++j) { BODY; }                              \
    }                                                                                        \
    T s = a[0];                                                                              \
    _Pragma("unroll") for (int j = 1; j < CH; ++j) s += a[j];                               \
    if (t < n) out[t] = *(uint32_t*)&s;                                                      \
  }

SINGLE(k_fma, float, seed + (float)(t + j), a[j] = __builtin_fmaf(a[j], k, seed))
SINGLE(k_add, float, seed + (float)(t + j), a[j] = a[j] + k)
SINGLE(k_log, float, seed + (float)(t + j), a[j] = __builtin_amdgcn_logf(a[j]))
SINGLE(k_exp, float, seed + (float)(t + j), a[j] = __builtin_amdgcn_exp2f(a[j]))
SINGLE(k_sqrt, float, seed + (float)(t + j), a[j] = __builtin_amdgcn_sqrtf(a[j]))
SINGLE(k_rcp, float, seed + (float)(t + j), a[j] = __builtin_amdgcn_rcpf(a[j]))
SINGLE(k_sin, float, seed + (float)(t + j), a[j] = __builtin_amdgcn_sinf(a[j]))
SINGLE(k_mulhi, uint32_t, seed + (uint32_t)(t * 7 + j), a[j] = __umulhi(a[j], k))
SINGLE(k_xor3, uint32_t, seed + (uint32_t)(t * 7 + j),
       asm volatile("v_bitop3_b32 %0, %0, %1, %2 bitop3:0x96" : "+v"(a[j]) : "v"(k), "v"(seed)))
SINGLE(k_addu, uint32_t, seed + (uint32_t)(t * 7 + j), asm volatile("v_add_u32 %0, %0, %1" : "+v"(a[j]) : "v"(k)))

#define PAIR(NAME, BODY2)                                                                    \
  __global__ __launch_bounds__(256) void NAME(float seed, float k, uint32_t* out, int n) {   \
    const int t = blockIdx.x * 256 + threadIdx.x;                                            \
    float a[CH];                                                                             \
    _Pragma("unroll") for (int j = 0; j < CH; ++j) a[j] = seed + (float)(t + j);            \
    for (int it = 0; it < ITER; ++it) {                                                      \
      _Pragma("unroll") for (int j = 0; j < CH; j += 2) {                                   \
        a[j] = __builtin_fmaf(a[j], k, seed);                                                \
        BODY2;                                                                               \
      }                                                                                      \
    }                                                                                        \
    float s = a[0];                                                                          \
    _Pragma("unroll") for (int j = 1; j < CH; ++j) s += a[j];                               \
    if (t < n) out[t] = __float_as_uint(s);                                                  \
  }

PAIR(k_fma_log, a[j + 1] = __builtin_amdgcn_logf(a[j + 1]))
PAIR(k_fma_sin, a[j + 1] = __builtin_amdgcn_sinf(a[j + 1]))
PAIR(k_fma_mulhi, {
  uint32_t u = __float_as_uint(a[j + 1]);
  u = __umulhi(u, 2654435761u);
  a[j + 1] = __uint_as_float(u);
})
PAIR(k_fma_xor3, {
  uint32_t u = __float_as_uint(a[j + 1]);
  asm volatile("v_bitop3_b32 %0, %0, %1, %2 bitop3:0x96" : "+v"(u) : "v"(t), "v"(it));
  a[j + 1] = __uint_as_float(u);
})

#define CHECK(call)                                                        \
  do {                                                                     \
    hipError_t e_ = (call);                                                \
    if (e_ != hipSuccess) {                                                \
      std::fprintf(stderr, "%s: %s\n", #call, hipGetErrorString(e_));      \
      return 1;                                                            \
    }                                                                      \
  } while (0)

int main() {
  int cus = 0;
  CHECK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, 0));
  const int blocks = cus * 8;  // 32 waves per CU, 8 per SIMD
  const int n = blocks * 256;  // one output word per thread
  uint32_t* out = nullptr;
  CHECK(hipMalloc(&out, sizeof(uint32_t) * (size_t)n));
  struct K {
    const char* name;
    void (*f)(float, float, uint32_t*, int);
    void (*g)(uint32_t, uint32_t, uint32_t*, int);
  };
  const std::vector<K> ks = {{"v_fma_f32", k_fma, nullptr},
                             {"v_add_f32", k_add, nullptr},
                             {"v_log_f32", k_log, nullptr},
                             {"v_exp_f32", k_exp, nullptr},
                             {"v_sqrt_f32", k_sqrt, nullptr},
                             {"v_rcp_f32", k_rcp, nullptr},
                             {"v_sin_f32", k_sin, nullptr},
                             {"v_mul_hi_u32", nullptr, k_mulhi},
                             {"v_bitop3_b32", nullptr, k_xor3},
                             {"v_add_u32", nullptr, k_addu},
                             {"half v_fma_f32, half v_log_f32", k_fma_log, nullptr},
                             {"half v_fma_f32, half v_sin_f32", k_fma_sin, nullptr},
                             {"half v_fma_f32, half v_mul_hi_u32", k_fma_mulhi, nullptr},
                             {"half v_fma_f32, half v_bitop3_b32", k_fma_xor3, nullptr}};
  hipEvent_t e0, e1;
  CHECK(hipEventCreate(&e0));
  CHECK(hipEventCreate(&e1));
  std::printf("{\"cus\": %d, \"blocks\": %d, \"waves\": %d, \"instructions_per_lane\": %d, \"results\": {", cus, blocks,
              n / 64, CH * ITER);
  for (size_t i = 0; i < ks.size(); ++i) {
    float best = 1e30f;
    for (int rep = 0; rep < 4; ++rep) {
      CHECK(hipEventRecord(e0, 0));
      if (ks[i].f)
        hipLaunchKernelGGL(ks[i].f, dim3(blocks), dim3(256), 0, 0, 1.25f, 0.999f, out, n);
      else
        hipLaunchKernelGGL(ks[i].g, dim3(blocks), dim3(256), 0, 0, 12345u, 2654435761u, out, n);
      CHECK(hipGetLastError());
      CHECK(hipEventRecord(e1, 0));
      CHECK(hipEventSynchronize(e1));
      float ms = 0;
      CHECK(hipEventElapsedTime(&ms, e0, e1));
      if (rep > 0 && ms < best) best = ms;
    }
    const double wave_insts = (double)(n / 64) * CH * ITER;
    std::printf("%s\"%s\": {\"ms\": %.4f, \"wave_insts_per_s\": %.4e}", i ? ", " : "", ks[i].name, best,
                wave_insts / (best * 1e-3));
  }
  std::printf("}}\n");
  CHECK(hipFree(out));
  return 0;
}
