// BF16 precision form of the fused score (Section III-B model, Section III-A
// Eq. 4, Section II-B Eq. 3): the same kernel as the FP32 form with the cross
// term on the BF16 matrix instructions. Launched by score_launch.
#include "score_device.h"

namespace fastron {

// ---------------------------------------------------------------------------
// BF16 MFMA form: with u = sqrt(gamma/2) p, t = 1 + ||u||^2 + ||u'||^2 - 2 u.u',
// the cross term -2 u.u' as bf16 products on v_mfma_f32_16x16x32_bf16 with
// FP32 accumulation. The support operand holds -2 u' as hi + mid + lo bf16
// parts (prepare kernel); the query side chooses the precision by which parts
// of u it pairs with them:
//   variant 0 (plain) : hi(u).hi(u'), with both norms taken from hi(u) and
//                       hi(u') as well, so that t is exactly 1 + the squared
//                       distance of the rounded points (up to float32
//                       rounding): the bf16 error then scales with the
//                       distance of the pair instead of with ||p|| ||p'||
//   variant 1 (split2): + mid(u).hi(u') + hi(u).mid(u')
//   variant 2 (split3): + lo(u).hi(u') + hi(u).lo(u') + mid(u).mid(u')
// The norms (computed in FP32) enter as three bf16 parts each against unit
// entries (exact to FP32 rounding), so the accumulator input is zero and no
// FP32 operand block has to be streamed besides the weights. Every t is
// clamped to t >= 1 (the squared distance to >= 0) before 1/t^2, so each K_RQ
// stays within (0, 1] whatever the cancellation in the BF16 cross term.
// ---------------------------------------------------------------------------
__device__ __forceinline__ unsigned short bf16_rne_d(float x) {
  uint32_t u = __float_as_uint(x);
  uint32_t r = u + 0x7fffu + ((u >> 16) & 1u);
  return (unsigned short)(r >> 16);
}
__device__ __forceinline__ float bf16_f(unsigned short h) { return __uint_as_float((uint32_t)h << 16); }

struct Split3 {
  unsigned short h, m, l;
};
__device__ __forceinline__ Split3 split3(float v) {
  Split3 s;
  s.h = bf16_rne_d(v);
  float r = v - bf16_f(s.h);
  s.m = bf16_rne_d(r);
  r -= bf16_f(s.m);
  s.l = bf16_rne_d(r);
  return s;
}

// Query-side value of k slot K (layout mirrors the prepared support operand);
// K is a compile-time constant, so only the variant (uniform) is decided at
// run time.
template <int K>
__device__ __forceinline__ unsigned short query_slot(int variant, const Split3& x, const Split3& y, const Split3& z,
                                                     const Split3& cq) {
  constexpr int grp = K / 3, comp = K % 3;
  const Split3& v = comp == 0 ? x : (comp == 1 ? y : z);
  if constexpr (grp == 0) return v.h;                        // against hi(u')
  else if constexpr (grp == 1) return variant >= 1 ? v.m : 0;  // against hi(u')
  else if constexpr (grp == 2) return variant >= 1 ? v.h : 0;  // against mid(u')
  else if constexpr (grp == 3) return variant >= 2 ? v.l : 0;  // against hi(u')
  else if constexpr (grp == 4) return variant >= 2 ? v.h : 0;  // against lo(u')
  else if constexpr (grp == 5) return variant >= 2 ? v.m : 0;  // against mid(u')
  else if constexpr (grp == 6) return comp == 0 ? cq.h : (comp == 1 ? cq.m : cq.l);  // against 1
  else if constexpr (grp == 7) return variant >= 1 ? 0x3f80 : 0;  // 1 against the parts of ||u'||^2
  else if constexpr (grp == 8) return variant == 0 ? 0x3f80 : 0;  // 1 against those of ||hi(u')||^2
  else return 0;
}

// The 8 slots 8 G .. 8 G + 7 that lane group G contributes to the operand.
template <int G>
__device__ __forceinline__ u16x8 query_group(int variant, const Split3& x, const Split3& y, const Split3& z,
                                             const Split3& cq) {
  return (u16x8){query_slot<8 * G + 0>(variant, x, y, z, cq), query_slot<8 * G + 1>(variant, x, y, z, cq),
                 query_slot<8 * G + 2>(variant, x, y, z, cq), query_slot<8 * G + 3>(variant, x, y, z, cq),
                 query_slot<8 * G + 4>(variant, x, y, z, cq), query_slot<8 * G + 5>(variant, x, y, z, cq),
                 query_slot<8 * G + 6>(variant, x, y, z, cq), query_slot<8 * G + 7>(variant, x, y, z, cq)};
}

// One wave stages 64 queries and scores them in 4 / QB passes of QB query
// blocks, so that only QB blocks' query operands (MM bf8 registers each) are
// resident while the support tiles stream.
template <int MM, typename R, bool RAT, int QB>
__global__ void __launch_bounds__(256) k_score_bf16(ChainArgs c, const float* __restrict__ q, int64_t N,
                                                     const char* __restrict__ blob, int64_t ntiles, int Mp,
                                                     float gamma, int variant, float* __restrict__ f,
                                                     int8_t* __restrict__ label) {
  __shared__ f4 lds[kWavesPerBlock][64][MM];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t qbase = ((int64_t)blockIdx.x * kWavesPerBlock + wave) * 64;
  stage_queries<MM, R>(c, q, N, gamma, qbase + lane, lds[wave]);
  __syncthreads();
  const int g = lane >> 4, col = lane & 15;
  const float f_const = reinterpret_cast<const float*>(blob)[0];
  const float* tiles = reinterpret_cast<const float*>(blob + kHeaderBytes);
  const int64_t tstride = tile_floats(Mp);
  const int64_t woff = tile_w_offset(Mp);
  const int64_t S_pad = ntiles * kTile;
  const u16x8* A16 = reinterpret_cast<const u16x8*>(blob + kHeaderBytes + ntiles * tstride * 4 +
                                                    S_pad * (int64_t)Mp * 16);
  const f4 zero = {0.f, 0.f, 0.f, 0.f};  // both norms arrive through the operands
  const float sg = sqrtf(0.5f * gamma);   // the prepare kernel's scale, computed the same way
#pragma unroll 1
  for (int h = 0; h < 4; h += QB) {
    bf8 B[QB][MM];
#pragma unroll
    for (int b = 0; b < QB; ++b)
#pragma unroll
      for (int m = 0; m < MM; ++m) {
        const f4 p = lds[wave][16 * (h + b) + col][m];
        const float ux = sg * p[0], uy = sg * p[1], uz = sg * p[2];
        const Split3 sx = split3(ux), sy = split3(uy), sz = split3(uz);
        // the squared norm as explicit fused multiply-adds (the prepare kernel's order)
        float nq;
        if (variant == 0) {
          const float hx = bf16_f(sx.h), hy = bf16_f(sy.h), hz = bf16_f(sz.h);
          nq = fmaf(hz, hz, fmaf(hy, hy, hx * hx));
        } else {
          nq = fmaf(uz, uz, fmaf(uy, uy, ux * ux));
        }
        const Split3 sc = split3(1.f + nq);
        // every group's slots are built with constant slot indices; each lane keeps its own group's
        const u16x8 u = g == 0 ? query_group<0>(variant, sx, sy, sz, sc)
                      : g == 1 ? query_group<1>(variant, sx, sy, sz, sc)
                      : g == 2 ? query_group<2>(variant, sx, sy, sz, sc)
                               : query_group<3>(variant, sx, sy, sz, sc);
        B[b][m] = __builtin_bit_cast(bf8, u);
      }
    float fpart[QB];
#pragma unroll
    for (int b = 0; b < QB; ++b) fpart[b] = 0.f;
    for (int64_t t = 0; t < ntiles; ++t) {
      const float* T = tiles + t * tstride;
      bf8 Av[MM];
#pragma unroll
      for (int m = 0; m < MM; ++m) Av[m] = __builtin_bit_cast(bf8, A16[(t * Mp + m) * 64 + lane]);
      const f4 W = *reinterpret_cast<const f4*>(T + woff + 4 * g);
#pragma unroll
      for (int b = 0; b < QB; ++b) {
        PairSum<RAT, true> ps;
#pragma unroll
        for (int m = 0; m < MM; ++m) ps.add(m, __builtin_amdgcn_mfma_f32_16x16x32_bf16(Av[m], B[b][m], zero, 0, 0, 0));
        fpart[b] = ps.finish(W, fpart[b]);
      }
    }
#pragma unroll
    for (int b = 0; b < QB; ++b) {
      float v = fpart[b];
      v += __shfl_xor(v, 16);
      v += __shfl_xor(v, 32);
      if (g == 0) write_result(qbase + 16 * (h + b) + col, N, v + f_const, f, label);
    }
  }
}

template <typename R>
static void launch_bf16_mm(const ChainArgs& c, int variant, bool rat, dim3 grid, hipStream_t s, const float* q,
                           int64_t N, const char* blob, int64_t nt, int Mp, float gamma, float* f, int8_t* label) {
#define FASTRON_BF_CASE(K)                                                                                      \
  case K:                                                                                                       \
    if (rat && qb == 2)                                                                                         \
      hipLaunchKernelGGL((k_score_bf16<K, R, true, 2>), grid, dim3(256), 0, s, c, q, N, blob, nt, Mp, gamma,    \
                         variant, f, label);                                                                    \
    else if (rat)                                                                                               \
      hipLaunchKernelGGL((k_score_bf16<K, R, true, 4>), grid, dim3(256), 0, s, c, q, N, blob, nt, Mp, gamma,    \
                         variant, f, label);                                                                    \
    else if (qb == 2)                                                                                           \
      hipLaunchKernelGGL((k_score_bf16<K, R, false, 2>), grid, dim3(256), 0, s, c, q, N, blob, nt, Mp, gamma,   \
                         variant, f, label);                                                                    \
    else                                                                                                        \
      hipLaunchKernelGGL((k_score_bf16<K, R, false, 4>), grid, dim3(256), 0, s, c, q, N, blob, nt, Mp, gamma,   \
                         variant, f, label);                                                                    \
    break;
  const int qb = (int)tune_get("score.bf16_blocks");
  switch (c.Mm) {
    FASTRON_BF_CASE(1) FASTRON_BF_CASE(2) FASTRON_BF_CASE(3) FASTRON_BF_CASE(4)
    FASTRON_BF_CASE(5) FASTRON_BF_CASE(6) FASTRON_BF_CASE(7) FASTRON_BF_CASE(8)
    FASTRON_BF_CASE(9) FASTRON_BF_CASE(10) FASTRON_BF_CASE(11) FASTRON_BF_CASE(12)
    FASTRON_BF_CASE(13) FASTRON_BF_CASE(14) FASTRON_BF_CASE(15) FASTRON_BF_CASE(16)
    default: break;
  }
#undef FASTRON_BF_CASE
}

void launch_score_bf16(const ChainArgs& c, int variant, bool rat, dim3 grid, hipStream_t s, const float* q,
                       int64_t N, const char* blob, int64_t nt, int Mp, float gamma, float* f, int8_t* label) {
  if (c.n >= kFp64Joints)
    launch_bf16_mm<double>(c, variant, rat, grid, s, q, N, blob, nt, Mp, gamma, f, label);
  else
    launch_bf16_mm<float>(c, variant, rat, grid, s, q, N, blob, nt, Mp, gamma, f, label);
}

}  // namespace fastron
