// Issue-rate probes behind the roofline of the scoring kernels.
//
// Each probe kernel runs one instruction kind in independent dependency
// chains (8 per lane for vector instructions, 4 accumulators for matrix
// instructions) so that issue, not latency, limits it, on a grid of
// `waves_per_simd` waves for every SIMD of the device. The host wrapper times
// the launch with HIP events and also reads the shader clock counter
// (s_memtime) against the constant 100 MHz clock (s_memrealtime) from inside
// the kernel, so that rates can be quoted in cycles per instruction at the
// clock the part actually ran.
//
// Kinds: 0 v_mul_f32, 1 v_fma_f32, 2 v_rcp_f32, 3 v_mfma_f32_16x16x4_f32,
// 4 v_mfma_f32_16x16x32_bf16, 5 one v_mfma_f32_16x16x4_f32 and 8 independent
// v_mul_f32 per round, 6 one v_mfma_f32_16x16x32_bf16 and 8 independent
// v_mul_f32 per round, 7 eight v_mul_f32 and one v_rcp_f32 per round.
// The vector instructions are written as inline assembly on registers only
// (no memory operands), so the compiler cannot merge, reorder or drop them.
#include <hip/hip_runtime.h>

#include <cstdint>

namespace {

typedef float f4p __attribute__((ext_vector_type(4)));
typedef __bf16 bf8p __attribute__((ext_vector_type(8)));

constexpr int kUnroll = 8;

#define P_MUL(x) asm volatile("v_mul_f32 %0, %0, %1" : "+v"(x) : "v"(k))
#define P_FMA(x) asm volatile("v_fma_f32 %0, %0, %1, %2" : "+v"(x) : "v"(k), "v"(c))
#define P_RCP(x) asm volatile("v_rcp_f32 %0, %0" : "+v"(x))
#define P_EIGHT(OP) \
  OP(x0);           \
  OP(x1);           \
  OP(x2);           \
  OP(x3);           \
  OP(x4);           \
  OP(x5);           \
  OP(x6);           \
  OP(x7)

struct ProbeClock {
  unsigned long long cycles;  // s_memtime delta of workgroup 0
  unsigned long long ticks;   // s_memrealtime delta (100 MHz) of workgroup 0
};

template <int KIND>
__global__ void __launch_bounds__(256) k_probe(float* __restrict__ out, ProbeClock* __restrict__ clk, int iters,
                                               float seed) {
  const unsigned long long c0 = __builtin_amdgcn_s_memtime();
  const unsigned long long t0 = __builtin_amdgcn_s_memrealtime();
  const float k = 1.0f + 1e-7f * seed, c = 1e-7f * seed;
  float x0 = seed + threadIdx.x, x1 = x0 + 1.f, x2 = x0 + 2.f, x3 = x0 + 3.f;
  float x4 = x0 + 4.f, x5 = x0 + 5.f, x6 = x0 + 6.f, x7 = x0 + 7.f;
  f4p a0 = {x0, x1, x2, x3}, a1 = a0, a2 = a0, a3 = a0;
  const f4p fa = {k, c, k, c};
  bf8p ba, bb;
  for (int e = 0; e < 8; ++e) {
    ba[e] = (__bf16)(k + e);
    bb[e] = (__bf16)(c + e);
  }
  const float fb = seed * 0.5f;
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      if constexpr (KIND == 0) {
        P_EIGHT(P_MUL);
      } else if constexpr (KIND == 1) {
        P_EIGHT(P_FMA);
      } else if constexpr (KIND == 2) {
        P_EIGHT(P_RCP);
      } else if constexpr (KIND == 3) {
        a0 = __builtin_amdgcn_mfma_f32_16x16x4f32(fa[0], fb, a0, 0, 0, 0);
        a1 = __builtin_amdgcn_mfma_f32_16x16x4f32(fa[1], fb, a1, 0, 0, 0);
        a2 = __builtin_amdgcn_mfma_f32_16x16x4f32(fa[2], fb, a2, 0, 0, 0);
        a3 = __builtin_amdgcn_mfma_f32_16x16x4f32(fa[3], fb, a3, 0, 0, 0);
      } else if constexpr (KIND == 4) {
        a0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ba, bb, a0, 0, 0, 0);
        a1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ba, bb, a1, 0, 0, 0);
        a2 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ba, bb, a2, 0, 0, 0);
        a3 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ba, bb, a3, 0, 0, 0);
      } else if constexpr (KIND == 5) {
        a0 = __builtin_amdgcn_mfma_f32_16x16x4f32(fa[0], fb, a0, 0, 0, 0);
        P_EIGHT(P_MUL);
      } else if constexpr (KIND == 6) {
        a0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ba, bb, a0, 0, 0, 0);
        P_EIGHT(P_MUL);
      } else {
        P_EIGHT(P_MUL);
        P_RCP(x0);
      }
    }
  }
  const float s = x0 + x1 + x2 + x3 + x4 + x5 + x6 + x7 + a0[0] + a1[1] + a2[2] + a3[3] + a0[3];
  // the results stay live through this store; its condition is never true for the seeds the host passes
  if (s == -1.2345f) out[blockIdx.x * blockDim.x + threadIdx.x] = s;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    clk->cycles = __builtin_amdgcn_s_memtime() - c0;
    clk->ticks = __builtin_amdgcn_s_memrealtime() - t0;
  }
}

// Plain device copy, 16 bytes per lane per iteration (grid-stride).
__global__ void __launch_bounds__(256) k_probe_copy(const float4* __restrict__ src, float4* __restrict__ dst,
                                                    int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) dst[i] = src[i];
}

}  // namespace

extern "C" {

// Instructions per lane per loop iteration of each kind (vector + matrix).
int probe_ops_per_iter(int kind, int* vector_ops, int* matrix_ops) {
  static const int v[8] = {8, 8, 8, 0, 0, 8, 8, 9};
  static const int m[8] = {0, 0, 0, 4, 4, 1, 1, 0};
  if (kind < 0 || kind > 7 || !vector_ops || !matrix_ops) return -1;
  *vector_ops = v[kind] * kUnroll;
  *matrix_ops = m[kind] * kUnroll;
  return 0;
}

// Runs probe `kind` on waves_per_simd * 4 * n_cu waves (256-thread
// workgroups) for `iters` loop iterations. Outputs: launch time (ms, HIP
// events on the null stream) and workgroup 0's shader-clock cycles and
// 100 MHz ticks. Returns 0, or -1 for bad arguments, -2 on a HIP error.
int probe_run(int kind, int waves_per_simd, int iters, double* ms, unsigned long long* cycles,
              unsigned long long* ticks, int* n_cu) {
  if (kind < 0 || kind > 7 || waves_per_simd < 1 || waves_per_simd > 8 || iters < 1 || !ms || !cycles || !ticks ||
      !n_cu)
    return -1;
  int dev = 0, ncu = 0;
  if (hipGetDevice(&dev) != hipSuccess) return -2;
  if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return -2;
  const int blocks = ncu * waves_per_simd;  // 4 waves per workgroup = one per SIMD
  float* out = nullptr;
  ProbeClock* clk = nullptr;
  if (hipMalloc(&out, (size_t)blocks * 256 * sizeof(float)) != hipSuccess) return -2;
  if (hipMalloc(&clk, sizeof(ProbeClock)) != hipSuccess) {
    (void)hipFree(out);
    return -2;
  }
  hipEvent_t e0, e1;
  (void)hipEventCreate(&e0);
  (void)hipEventCreate(&e1);
  auto launch = [&](int it) {
    switch (kind) {
      case 0: hipLaunchKernelGGL(k_probe<0>, dim3(blocks), dim3(256), 0, 0, out, clk, it, 1.5f); break;
      case 1: hipLaunchKernelGGL(k_probe<1>, dim3(blocks), dim3(256), 0, 0, out, clk, it, 1.5f); break;
      case 2: hipLaunchKernelGGL(k_probe<2>, dim3(blocks), dim3(256), 0, 0, out, clk, it, 1.5f); break;
      case 3: hipLaunchKernelGGL(k_probe<3>, dim3(blocks), dim3(256), 0, 0, out, clk, it, 1.5f); break;
      case 4: hipLaunchKernelGGL(k_probe<4>, dim3(blocks), dim3(256), 0, 0, out, clk, it, 1.5f); break;
      case 5: hipLaunchKernelGGL(k_probe<5>, dim3(blocks), dim3(256), 0, 0, out, clk, it, 1.5f); break;
      case 6: hipLaunchKernelGGL(k_probe<6>, dim3(blocks), dim3(256), 0, 0, out, clk, it, 1.5f); break;
      default: hipLaunchKernelGGL(k_probe<7>, dim3(blocks), dim3(256), 0, 0, out, clk, it, 1.5f); break;
    }
  };
  launch(iters / 8 + 1);  // warm-up
  (void)hipEventRecord(e0, 0);
  launch(iters);
  (void)hipEventRecord(e1, 0);
  hipError_t err = hipEventSynchronize(e1);
  float t = 0.f;
  if (err == hipSuccess) err = hipEventElapsedTime(&t, e0, e1);
  ProbeClock h{0, 0};
  if (err == hipSuccess) err = hipMemcpy(&h, clk, sizeof(h), hipMemcpyDeviceToHost);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipFree(out);
  (void)hipFree(clk);
  if (err != hipSuccess) return -2;
  *ms = t;
  *cycles = h.cycles;
  *ticks = h.ticks;
  *n_cu = ncu;
  return 0;
}

// Device-to-device copy of `bytes` (a multiple of 16) with the probe copy
// kernel, `reps` timed launches; *ms = mean time per copy.
int probe_copy(const void* src, void* dst, int64_t bytes, int reps, double* ms) {
  if (!src || !dst || bytes <= 0 || bytes % 16 != 0 || reps < 1 || !ms) return -1;
  int dev = 0, ncu = 0;
  if (hipGetDevice(&dev) != hipSuccess) return -2;
  if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return -2;
  const int64_t n = bytes / 16;
  const unsigned blocks = (unsigned)(ncu * 16);
  hipEvent_t e0, e1;
  (void)hipEventCreate(&e0);
  (void)hipEventCreate(&e1);
  hipLaunchKernelGGL(k_probe_copy, dim3(blocks), dim3(256), 0, 0, static_cast<const float4*>(src),
                     static_cast<float4*>(dst), n);
  (void)hipEventRecord(e0, 0);
  for (int r = 0; r < reps; ++r)
    hipLaunchKernelGGL(k_probe_copy, dim3(blocks), dim3(256), 0, 0, static_cast<const float4*>(src),
                       static_cast<float4*>(dst), n);
  (void)hipEventRecord(e1, 0);
  hipError_t err = hipEventSynchronize(e1);
  float t = 0.f;
  if (err == hipSuccess) err = hipEventElapsedTime(&t, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (err != hipSuccess) return -2;
  *ms = t / reps;
  return 0;
}

}  // extern "C"
