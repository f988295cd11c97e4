// Device-side pieces shared by the scoring kernels (single-model FP32 and
// BF16, batched): query staging (fused FK), the per-pair K_RQ sums, the FP32
// MFMA wave loop and result writing. Included by score.hip, score_bf16.hip
// and batch.hip only.
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

// Sum over a pair's control points of 1/t^2 for a lane's 4 (support, query)
// pairs (component r of each MFMA result: support row r), fed one point at a
// time in point order; finish() adds sum_r W[r] * sum_m 1/t_{m,r}^2 to acc.
// Two forms:
//   RAT = false: r = 1/t with the reciprocal saturated at 1 (t >= 1; this also
//                guards against cancellation), then s += r^2: one
//                quarter-rate reciprocal and one FMA per value.
//   RAT = true : the sum as one running fraction n/e with v_m = t_m^2,
//                e <- e v_m and n <- n v_m + e (n = 1, e = v_0 at the start),
//                then one reciprocal of e per pair: three full-rate
//                operations per value. All terms are positive, so the
//                fraction is as accurate as the direct sum; the caller takes
//                this form only when a bound on t keeps e = prod t_m^2 inside
//                the normal FP32 range and t away from 0 (rational_sum_ok).
// CLAMP: t is first raised to at least 1, i.e. the squared distance to at
// least 0 (K_RQ <= 1, Eq. 3), one more operation per value (v_med3_f32 with
// 1 and 3e38: the same clamp for every t up to 3e38; IEEE-mode fmaxf would
// cost a canonicalising max on top). The BF16 forms take it: their cross
// term can be off by about 2^-8 gamma ||p|| ||p'||, so cancellation could
// otherwise push t of a near-coincident pair well below 1. In the FP32 form
// t is off by at most a few units of 2^-24 t, so the unclamped running
// fraction stays within rounding of the clamped one and the saturated
// reciprocal clamps at no cost.
template <bool RAT, bool CLAMP = false>
struct PairSum {
  float n[4] = {1.f, 1.f, 1.f, 1.f};  // RAT: numerators;   else: the sums
  float e[4] = {0.f, 0.f, 0.f, 0.f};  // RAT: denominators; else: unused

  __device__ __forceinline__ PairSum() {
    if constexpr (!RAT) n[0] = n[1] = n[2] = n[3] = 0.f;
  }
  __device__ __forceinline__ void add(int m, const f4& d) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const float t = CLAMP ? __builtin_amdgcn_fmed3f(d[r], 1.0f, 3.0e38f) : d[r];
      if constexpr (RAT) {
        const float v = t * t;
        if (m == 0) {
          e[r] = v;
        } else {
          n[r] = fmaf(n[r], v, e[r]);
          e[r] *= v;
        }
      } else {
        const float x = CLAMP ? __builtin_amdgcn_rcpf(t) : rcp_sat(t);
        n[r] = fmaf(x, x, n[r]);
      }
    }
  }
  __device__ __forceinline__ float finish(const f4& W, float acc) const {
    float s[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      if constexpr (RAT) s[r] = n[r] * __builtin_amdgcn_rcpf(e[r]);
      else s[r] = n[r];
    }
    return fmaf(W[0], s[0], fmaf(W[1], s[1], fmaf(W[2], s[2], fmaf(W[3], s[3], acc))));
  }
};

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
// PAIRED: interleave the MFMAs of two query blocks (more registers in flight;
// the persistent batched kernel, which holds more state, leaves it off).
template <int MM, int QB, bool RAT, bool PAIRED>
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
    // query blocks in pairs: each point's two MFMAs are issued back to back,
    // so one block's result is in flight while the other's is consumed
#pragma unroll
    for (int b = 0; b < QB; b += 2) {
      if (PAIRED && b + 1 < QB) {
        PairSum<RAT> p0, p1;
#pragma unroll
        for (int m = 0; m < MM; ++m) {
          const f4 d0 = __builtin_amdgcn_mfma_f32_16x16x4f32(Av[m >> 2][m & 3], B[b][m], Cv[m], 0, 0, 0);
          const f4 d1 = __builtin_amdgcn_mfma_f32_16x16x4f32(Av[m >> 2][m & 3], B[b + 1][m], Cv[m], 0, 0, 0);
          p0.add(m, d0);
          p1.add(m, d1);
        }
        fpart[b] = p0.finish(W, fpart[b]);
        fpart[b + 1] = p1.finish(W, fpart[b + 1]);
      } else {
#pragma unroll
        for (int h = b; h < b + 2 && h < QB; ++h) {
          PairSum<RAT> ps;
#pragma unroll
          for (int m = 0; m < MM; ++m)
            ps.add(m, __builtin_amdgcn_mfma_f32_16x16x4f32(Av[m >> 2][m & 3], B[h][m], Cv[m], 0, 0, 0));
          fpart[h] = ps.finish(W, fpart[h]);
        }
      }
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

// BF16 form launcher (score_bf16.hip): one kernel per moving-point count,
// FK precision and summation form; variant = FASTRON_BF16_* >> 4.
void launch_score_bf16(const ChainArgs& c, int variant, bool rat, dim3 grid, hipStream_t s, const float* q,
                       int64_t N, const char* blob, int64_t nt, int Mp, float gamma, float* f, int8_t* label);

}  // namespace fastron
