// Device-side pieces shared by the single-model and the batched scoring
// kernels: query staging (fused FK), the FP32 MFMA wave loop and result
// writing. Included by score.hip and batch.hip only.
#pragma once

#include "fastron_internal.h"
#include "model_layout.h"

namespace fastron {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));

// 1/t saturated to [0, 1]: the reciprocal's clamp output modifier.
__device__ __forceinline__ float rcp_sat(float t) {
  return __builtin_amdgcn_fmed3f(__builtin_amdgcn_rcpf(t), 0.0f, 1.0f);
}

constexpr int kWavesPerBlock = 4;

// Stage this wave's 64 query control points in LDS as (x, y, z, c_q), slot-major.
template <int MM, typename R>
__device__ __forceinline__ void stage_queries(const ChainArgs& c, const float* __restrict__ q, int64_t N, float gamma,
                                              int64_t j, f4 (*lds)[MM]) {
  const int lane = threadIdx.x & 63;
  float qv[FASTRON_MAX_JOINTS];
#pragma unroll
  for (int i = 0; i < FASTRON_MAX_JOINTS; ++i)
    if (i < c.n) qv[i] = (j < N) ? q[j * c.n + i] : 0.0f;
  const float half_g = 0.5f * gamma;
  fk_walk<R>(c, qv, [&](int m, float x, float y, float z) {
    const int slot = c.slot[m];
    if (slot < 0) return;
    f4 v = {x, y, z, 1.0f + half_g * (x * x + y * y + z * z)};
    lds[lane][slot] = v;
  });
}

__device__ __forceinline__ void write_result(int64_t j, int64_t N, float v, float* __restrict__ f,
                                             int8_t* __restrict__ label) {
  if (j < N) {
    if (f) f[j] = v;
    if (label) label[j] = (v >= 0.0f) ? (int8_t)1 : (int8_t)-1;
  }
}

// One wave scores the 16 * QB queries staged in `lds` (rows 16 b + col) against
// `ntiles` support tiles; queries with index >= qend are not written.
template <int MM, int QB>
__device__ __forceinline__ void wave_score_fp32(const f4 (*lds)[MM], const float* __restrict__ tiles, int64_t ntiles,
                                                int Mp, float f_const, int64_t qbase, int64_t qend,
                                                float* __restrict__ f, int8_t* __restrict__ label) {
  const int lane = threadIdx.x & 63;
  const int g = lane >> 4, col = lane & 15;
  float B[QB][MM];
#pragma unroll
  for (int b = 0; b < QB; ++b)
#pragma unroll
    for (int m = 0; m < MM; ++m) B[b][m] = lds[16 * b + col][m][g];
  const int64_t tstride = tile_floats(Mp);
  const int64_t coff = tile_c_offset(Mp), woff = tile_w_offset(Mp);
  float fpart[QB];
#pragma unroll
  for (int b = 0; b < QB; ++b) fpart[b] = 0.f;
  constexpr int MV = (MM + 3) / 4;
  for (int64_t t = 0; t < ntiles; ++t) {
    const float* T = tiles + t * tstride;
    f4 Av[MV];
#pragma unroll
    for (int i = 0; i < MV; ++i) Av[i] = *reinterpret_cast<const f4*>(T + lane * Mp + 4 * i);
    f4 Cv[MM];
#pragma unroll
    for (int m = 0; m < MM; ++m) Cv[m] = *reinterpret_cast<const f4*>(T + coff + (g * Mp + m) * 4);
    const f4 W = *reinterpret_cast<const f4*>(T + woff + 4 * g);
#pragma unroll
    for (int b = 0; b < QB; ++b) {
      float a0 = 0.f, a1 = 0.f, a2 = 0.f, a3 = 0.f;
#pragma unroll
      for (int m = 0; m < MM; ++m) {
        const f4 d = __builtin_amdgcn_mfma_f32_16x16x4f32(Av[m >> 2][m & 3], B[b][m], Cv[m], 0, 0, 0);
        const float r0 = rcp_sat(d[0]), r1 = rcp_sat(d[1]), r2 = rcp_sat(d[2]), r3 = rcp_sat(d[3]);
        a0 = fmaf(r0, r0, a0);
        a1 = fmaf(r1, r1, a1);
        a2 = fmaf(r2, r2, a2);
        a3 = fmaf(r3, r3, a3);
      }
      fpart[b] = fmaf(W[0], a0, fmaf(W[1], a1, fmaf(W[2], a2, fmaf(W[3], a3, fpart[b]))));
    }
  }
#pragma unroll
  for (int b = 0; b < QB; ++b) {
    float v = fpart[b];
    v += __shfl_xor(v, 16);
    v += __shfl_xor(v, 32);
    if (g == 0) write_result(qbase + 16 * b + col, qend, v + f_const, f, label);
  }
}

}  // namespace fastron
