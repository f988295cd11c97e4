// Fused FK-kernel score f(q) = sum_i alpha_i K_FK(S_i, q) and its sign
// (Section III-B model, Section III-A Eq. 4, Section II-B Eq. 3).
//
// Per query q, support s and moving control point m the kernel needs
//   t = 1 + gamma/2 ||p - p'||^2 = c_q + c_s - gamma p.p'
// with c_q = 1 + gamma/2 ||p||^2 and c_s = gamma/2 ||p'||^2, then K_RQ = 1/t^2.
// The nonlinearity acts on each control point's own distance, so the
// contraction is M separate 3-deep dot products, not one 3M-deep one. With
// supports as rows and queries as columns, one v_mfma_f32_16x16x4_f32 computes
// t for 16 supports x 16 queries of one control point:
//   A[s] = (-gamma x', -gamma y', -gamma z', 1)   (prepared support operand)
//   B[q] = (x, y, z, c_q)                        (query FK, computed here)
//   C[s][q] = c_s                                (per-row constant)
// Each lane then turns its 4 outputs into 1/t^2 with one reciprocal (its
// clamp modifier saturates at 1, i.e. t >= 1, which guards against
// cancellation) and one FMA, accumulating over m; alpha_s / M weights the sum
// once per (s, q) and the four lane groups are reduced with shuffles at the
// end. Points fixed to the base contribute exactly 1 per pair and arrive as
// the constant f_const.
#include <cmath>

#include "score_device.h"

namespace fastron {

// ---------------------------------------------------------------------------
// FP32 MFMA form (default): one wave per 64 queries.
// ---------------------------------------------------------------------------
template <int MM, typename R>
__global__ void __launch_bounds__(256) k_score_mfma(ChainArgs c, const float* __restrict__ q, int64_t N,
                                                     const char* __restrict__ blob, int64_t ntiles, int Mp,
                                                     float gamma, float* __restrict__ f,
                                                     int8_t* __restrict__ label) {
  __shared__ f4 lds[kWavesPerBlock][64][MM];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t qbase = ((int64_t)blockIdx.x * kWavesPerBlock + wave) * 64;
  stage_queries<MM, R>(c, q, N, gamma, qbase + lane, lds[wave]);
  __syncthreads();
  const float f_const = reinterpret_cast<const float*>(blob)[0];
  const float* tiles = reinterpret_cast<const float*>(blob + kHeaderBytes);
  wave_score_fp32<MM, 4>(lds[wave], tiles, ntiles, Mp, f_const, qbase, N, f, label);
}

// ---------------------------------------------------------------------------
// BF16 MFMA form: the cross term -gamma p.p' as bf16 products on
// v_mfma_f32_16x16x32_bf16 with FP32 accumulation. The support operand holds
// -gamma p' as hi + mid + lo bf16 parts (prepare kernel); the query side
// chooses the precision by which parts of p it pairs with them:
//   variant 0 (plain) : hi(p).hi(p')
//   variant 1 (split2): + mid(p).hi(p') + hi(p).mid(p')
//   variant 2 (split3): + lo(p).hi(p') + hi(p).lo(p') + mid(p).mid(p')
// c_q enters through three bf16 parts against unit entries (exact to FP32
// rounding), c_s through the FP32 accumulator input.
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

// Query-side value of k slot `k` (layout mirrors the prepared support operand).
__device__ __forceinline__ unsigned short query_slot(int k, int variant, const Split3& x, const Split3& y,
                                                     const Split3& z, const Split3& cq) {
  const int grp = k / 3, comp = k % 3;
  const Split3& v = comp == 0 ? x : (comp == 1 ? y : z);
  switch (grp) {
    case 0: return v.h;                          // against hi(p')
    case 1: return variant >= 1 ? v.m : 0;       // against hi(p')
    case 2: return variant >= 1 ? v.h : 0;       // against mid(p')
    case 3: return variant >= 2 ? v.l : 0;       // against hi(p')
    case 4: return variant >= 2 ? v.h : 0;       // against lo(p')
    case 5: return variant >= 2 ? v.m : 0;       // against mid(p')
    case 6: return comp == 0 ? cq.h : (comp == 1 ? cq.m : cq.l);  // against 1
    default: return 0;
  }
}

template <int MM, typename R>
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
  bf8 B[4][MM];
#pragma unroll
  for (int b = 0; b < 4; ++b)
#pragma unroll
    for (int m = 0; m < MM; ++m) {
      const f4 p = lds[wave][16 * b + col][m];
      const Split3 sx = split3(p[0]), sy = split3(p[1]), sz = split3(p[2]), sc = split3(p[3]);
      u16x8 u;
#pragma unroll
      for (int e = 0; e < 8; ++e) u[e] = query_slot(8 * g + e, variant, sx, sy, sz, sc);
      B[b][m] = __builtin_bit_cast(bf8, u);
    }

  const float f_const = reinterpret_cast<const float*>(blob)[0];
  const float* tiles = reinterpret_cast<const float*>(blob + kHeaderBytes);
  const int64_t tstride = tile_floats(Mp);
  const int64_t coff = tile_c_offset(Mp), woff = tile_w_offset(Mp);
  const int64_t S_pad = ntiles * kTile;
  const u16x8* A16 = reinterpret_cast<const u16x8*>(blob + kHeaderBytes + ntiles * tstride * 4 +
                                                    S_pad * (int64_t)Mp * 16);
  float fpart[4] = {0.f, 0.f, 0.f, 0.f};
  for (int64_t t = 0; t < ntiles; ++t) {
    const float* T = tiles + t * tstride;
    bf8 Av[MM];
#pragma unroll
    for (int m = 0; m < MM; ++m) Av[m] = __builtin_bit_cast(bf8, A16[(t * Mp + m) * 64 + lane]);
    f4 Cv[MM];
#pragma unroll
    for (int m = 0; m < MM; ++m) Cv[m] = *reinterpret_cast<const f4*>(T + coff + (g * Mp + m) * 4);
    const f4 W = *reinterpret_cast<const f4*>(T + woff + 4 * g);
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      float a0 = 0.f, a1 = 0.f, a2 = 0.f, a3 = 0.f;
#pragma unroll
      for (int m = 0; m < MM; ++m) {
        const f4 d = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Av[m], B[b][m], Cv[m], 0, 0, 0);
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
  for (int b = 0; b < 4; ++b) {
    float v = fpart[b];
    v += __shfl_xor(v, 16);
    v += __shfl_xor(v, 32);
    if (g == 0) write_result(qbase + 16 * b + col, N, v + f_const, f, label);
  }
}

// ---------------------------------------------------------------------------
// VALU form: one query per lane, the cross term as three FMAs against
// wave-uniform support operands. Same result, no MFMA; kept as the baseline
// that the MFMA forms are measured against.
// ---------------------------------------------------------------------------
template <int MM, typename R>
__global__ void __launch_bounds__(256) k_score_valu(ChainArgs c, const float* __restrict__ q, int64_t N,
                                                     const char* __restrict__ blob, int64_t ntiles, int Mp,
                                                     float gamma, float* __restrict__ f,
                                                     int8_t* __restrict__ label) {
  __shared__ f4 lds[kWavesPerBlock][64][MM];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t j = ((int64_t)blockIdx.x * kWavesPerBlock + wave) * 64 + lane;
  stage_queries<MM, R>(c, q, N, gamma, j, lds[wave]);
  __syncthreads();
  f4 P[MM];
#pragma unroll
  for (int m = 0; m < MM; ++m) P[m] = lds[wave][lane][m];
  const float f_const = reinterpret_cast<const float*>(blob)[0];
  const float* tiles = reinterpret_cast<const float*>(blob + kHeaderBytes);
  const int64_t tstride = tile_floats(Mp);
  const int64_t woff = tile_w_offset(Mp);
  const f4* V = reinterpret_cast<const f4*>(blob + kHeaderBytes + ntiles * tstride * 4);
  float acc_f = 0.f;
  const int64_t S_pad = ntiles * kTile;
  for (int64_t s = 0; s < S_pad; ++s) {
    const float w = tiles[(s >> 4) * tstride + woff + (s & 15)];
    float acc = 0.f;
#pragma unroll
    for (int m = 0; m < MM; ++m) {
      const f4 v = V[s * Mp + m];
      const float t = fmaf(v[0], P[m][0], fmaf(v[1], P[m][1], fmaf(v[2], P[m][2], P[m][3] + v[3])));
      const float r = rcp_sat(t);
      acc = fmaf(r, r, acc);
    }
    acc_f = fmaf(w, acc, acc_f);
  }
  write_result(j, N, acc_f + f_const, f, label);
}

// All control points fixed to the base: K_FK = 1 for every pair.
__global__ void __launch_bounds__(256) k_score_const(const char* __restrict__ blob, int64_t N, float* __restrict__ f,
                                                      int8_t* __restrict__ label) {
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  write_result(j, N, reinterpret_cast<const float*>(blob)[0], f, label);
}

// ---------------------------------------------------------------------------
// Host dispatch over the number of moving points and the FK precision.
// ---------------------------------------------------------------------------
template <int MM, typename R>
static void launch_one(uint32_t kind, int variant, dim3 grid, hipStream_t s, const ChainArgs& c, const float* q,
                       int64_t N, const char* blob, int64_t nt, int Mp, float gamma, float* f, int8_t* label) {
  if (kind == FASTRON_SCORE_BF16)
    hipLaunchKernelGGL((k_score_bf16<MM, R>), grid, dim3(256), 0, s, c, q, N, blob, nt, Mp, gamma, variant, f, label);
  else if (kind == FASTRON_SCORE_VALU)
    hipLaunchKernelGGL((k_score_valu<MM, R>), grid, dim3(256), 0, s, c, q, N, blob, nt, Mp, gamma, f, label);
  else
    hipLaunchKernelGGL((k_score_mfma<MM, R>), grid, dim3(256), 0, s, c, q, N, blob, nt, Mp, gamma, f, label);
}

template <typename R>
static void launch_mm(int Mm, uint32_t kind, int variant, dim3 grid, hipStream_t s, const ChainArgs& c,
                      const float* q, int64_t N, const char* blob, int64_t nt, int Mp, float gamma, float* f,
                      int8_t* label) {
#define FASTRON_MM_CASE(K) \
  case K: launch_one<K, R>(kind, variant, grid, s, c, q, N, blob, nt, Mp, gamma, f, label); break;
  switch (Mm) {
    FASTRON_MM_CASE(1) FASTRON_MM_CASE(2) FASTRON_MM_CASE(3) FASTRON_MM_CASE(4)
    FASTRON_MM_CASE(5) FASTRON_MM_CASE(6) FASTRON_MM_CASE(7) FASTRON_MM_CASE(8)
    FASTRON_MM_CASE(9) FASTRON_MM_CASE(10) FASTRON_MM_CASE(11) FASTRON_MM_CASE(12)
    FASTRON_MM_CASE(13) FASTRON_MM_CASE(14) FASTRON_MM_CASE(15) FASTRON_MM_CASE(16)
    default: break;
  }
#undef FASTRON_MM_CASE
}

// Shared by the single-model and batched entry points.
fastron_status score_launch(const ChainArgs& c, const fastron_model* model, const float* q, int64_t N, float* f,
                            int8_t* label, uint32_t flags, hipStream_t s) {
  const uint32_t kind = flags & 3u;
  const int variant = (int)((flags >> 4) & 3u);
  const int64_t nt = ntiles_of(model->S);
  const int Mp = mp_of(c.M);
  const int64_t blocks = (N + 64 * kWavesPerBlock - 1) / (64 * kWavesPerBlock);
  FASTRON_CHECK(blocks <= INT32_MAX, "N too large");
  const char* blob = static_cast<const char*>(model->data);
  if (c.Mm == 0) {
    hipLaunchKernelGGL(k_score_const, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s, blob, N, f, label);
  } else if (c.n >= kFp64Joints) {
    launch_mm<double>(c.Mm, kind, variant, dim3((unsigned)blocks), s, c, q, N, blob, nt, Mp, model->gamma, f, label);
  } else {
    launch_mm<float>(c.Mm, kind, variant, dim3((unsigned)blocks), s, c, q, N, blob, nt, Mp, model->gamma, f, label);
  }
  FASTRON_HIP(hipGetLastError());
  return FASTRON_OK;
}

}  // namespace fastron

using namespace fastron;

static fastron_status check_score_args(const ChainArgs& c, const fastron_model* model, const float* q, int64_t N,
                                       float* f, int8_t* label, uint32_t flags) {
  FASTRON_CHECK(model != nullptr, "model is NULL");
  FASTRON_CHECK(model->data != nullptr && fastron::aligned(model->data, 256), "model->data must be 256-byte aligned");
  FASTRON_CHECK(model->S >= 0, "model->S < 0");
  FASTRON_CHECK(model->M == c.M, "model was prepared for M = %d, control points have M = %d", model->M, c.M);
  FASTRON_CHECK(model->bytes >= fastron::model_bytes(model->S, c.M), "model->bytes too small for S = %lld",
                (long long)model->S);
  FASTRON_CHECK(std::isfinite(model->gamma) && model->gamma > 0.f, "model->gamma must be finite and > 0");
  FASTRON_CHECK(N >= 0, "N = %lld < 0", (long long)N);
  FASTRON_CHECK(N == 0 || q != nullptr, "q is NULL");
  FASTRON_CHECK(N == 0 || f != nullptr || label != nullptr, "f and label are both NULL");
  FASTRON_CHECK((flags & ~0x33u) == 0 && (flags & 3u) != 3u, "unknown flags 0x%x", flags);
  FASTRON_CHECK(((flags >> 4) & 3u) <= 2u, "unknown BF16 variant");
  return FASTRON_OK;
}

extern "C" {

fastron_status fastron_fk_score_prepared(const fastron_chain* chain, const fastron_cpoints* cp,
                                         const fastron_model* model, const float* q, int64_t N, float* f,
                                         int8_t* label, uint32_t flags, void* stream) {
  clear_error();
  ChainArgs c;
  fastron_status st = pack_chain(chain, cp, &c, true);
  if (st != FASTRON_OK) return st;
  st = check_score_args(c, model, q, N, f, label, flags);
  if (st != FASTRON_OK) return st;
  if (N == 0) return FASTRON_OK;
  return score_launch(c, model, q, N, f, label, flags, as_stream(stream));
}

fastron_status fastron_fk_score(const fastron_chain* chain, const fastron_cpoints* cp, const float* support_q,
                                const float* alpha, int64_t S, float gamma, const float* q, int64_t N, float* f,
                                int8_t* label, uint32_t flags, void* stream) {
  clear_error();
  ChainArgs c;
  fastron_status st = pack_chain(chain, cp, &c, true);
  if (st != FASTRON_OK) return st;
  FASTRON_CHECK(S >= 0, "S = %lld < 0", (long long)S);
  FASTRON_CHECK(S == 0 || (support_q && alpha), "support_q and alpha must be non-NULL when S > 0");
  FASTRON_CHECK(std::isfinite(gamma) && gamma > 0.f, "gamma must be finite and > 0");
  fastron_model probe{S, c.M, gamma, reinterpret_cast<void*>(256), fastron::model_bytes(S, c.M)};
  st = check_score_args(c, &probe, q, N, f, label, flags);
  if (st != FASTRON_OK) return st;
  if (N == 0) return FASTRON_OK;
  hipStream_t s = as_stream(stream);
  const int64_t bytes = fastron::model_bytes(S, c.M);
  void* blob = nullptr;
  FASTRON_HIP(hipMallocAsync(&blob, (size_t)bytes, s));
  fastron_model model{S, c.M, gamma, blob, bytes};
  st = fastron_support_prep(chain, cp, support_q, alpha, S, gamma, &model, stream);
  if (st == FASTRON_OK) st = score_launch(c, &model, q, N, f, label, flags, s);
  hipError_t e = hipFreeAsync(blob, s);
  if (st != FASTRON_OK) return st;
  if (e != hipSuccess) return fail(FASTRON_EHIP, "hipFreeAsync failed: %s", hipGetErrorString(e));
  return FASTRON_OK;
}

}  // extern "C"
