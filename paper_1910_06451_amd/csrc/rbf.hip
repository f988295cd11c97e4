// Fastron model with the rational quadratic kernel of Eq. 3 applied to the
// configurations themselves -- the kernel the paper compares the FK kernel
// with (Section II-B, Eq. 3; Section IV): f(x) = sum_s alpha_s K_RQ(x_s, x) for
// joint vectors of n <= 16 coordinates, and its sign.
//
// Per (query, support) pair t = 1 + gamma/2 ||x - x'||^2 = c_q + c_s - gamma x . x'
// with c_q = 1 + gamma/2 ||x||^2 and c_s = gamma/2 ||x'||^2: an (n + 1)-deep
// contraction of A[s] = (-gamma x', 1) with B[q] = (x, c_q) plus the per-support
// constant, done in KS = ceil((n + 1) / 4) steps of v_mfma_f32_16x16x4_f32
// (supports as rows, queries as columns, c_s as the first accumulator). Then
// the reciprocal saturated at 1 (t >= 1; it guards against cancellation), its
// square, and alpha_s; the four lane groups are reduced with shuffles.
//
// Prepared tile of 16 supports (floats): A[KS][64] (lane l: support l % 16,
// coordinate 4 c + l / 16: -gamma x'_k for k < n, 1 for k = n, else 0), then
// C[16] = c_s and W[16] = alpha_s. Padded rows hold A = (0, .., 1, 0, ..),
// C = 0, W = 0: t = c_q >= 1 and a zero weight.
#include <cmath>

#include "fastron_internal.h"

namespace fastron {

typedef float rf4 __attribute__((ext_vector_type(4)));

__host__ __device__ constexpr int64_t rbf_tile_floats(int KS) { return 64 * KS + 32; }

__device__ __forceinline__ float rbf_rcp_sat(float t) {
  return __builtin_amdgcn_fmed3f(__builtin_amdgcn_rcpf(t), 0.0f, 1.0f);
}

// One thread per padded support row.
__global__ void __launch_bounds__(256) k_rbf_prep(const float* __restrict__ sx, const float* __restrict__ alpha,
                                                   int64_t S, int n, int KS, int64_t ntiles, float gamma,
                                                   float* __restrict__ tiles) {
  const int64_t s = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (s >= ntiles * 16) return;
  const int64_t tile = s / 16;
  const int sl = (int)(s % 16);
  float* T = tiles + tile * rbf_tile_floats(KS);
  const bool real = s < S;
  float nrm = 0.f;
  for (int k = 0; k < 4 * KS; ++k) {
    float v = 0.f;
    if (k < n && real) {
      const float x = sx[s * n + k];
      v = -gamma * x;
      nrm = fmaf(x, x, nrm);
    } else if (k == n) {
      v = 1.f;
    }
    T[(k >> 2) * 64 + (k & 3) * 16 + sl] = v;
  }
  T[64 * KS + sl] = real ? 0.5f * gamma * nrm : 0.f;
  T[64 * KS + 16 + sl] = real ? alpha[s] : 0.f;
}

// One wave scores QB = 4 blocks of 16 queries against every tile. Each lane
// reads the coordinates it feeds the contraction (and its query's norm)
// straight from the query array once; the tile loop then touches only the
// tiles. (Eight blocks per wave measured within 5 % at 1,000,000 queries and
// slower at small N.)
template <int KS>
__global__ void __launch_bounds__(256) k_score_rbf(const float* __restrict__ q, int64_t N, int n, float gamma,
                                                    const float* __restrict__ tiles, int64_t ntiles,
                                                    float* __restrict__ f, int8_t* __restrict__ label) {
  constexpr int QB = 4;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t qbase = ((int64_t)blockIdx.x * 4 + wave) * (16 * QB);
  const int g = lane >> 4, col = lane & 15;
  float B[QB][KS];
#pragma unroll
  for (int b = 0; b < QB; ++b) {
    const int64_t j = qbase + 16 * b + col;
    float nrm = 0.f;
#pragma unroll
    for (int c = 0; c < KS; ++c) B[b][c] = 0.f;
    if (j < N) {
#pragma unroll
      for (int k = 0; k < 4 * KS; ++k) {
        if (k < n) {
          const float v = q[j * n + k];
          nrm = fmaf(v, v, nrm);
          if ((k & 3) == g) B[b][k >> 2] = v;
        }
      }
    }
    // entry n of B is c_q (1 past the end of the queries, whose outputs are not written)
    const float cq = 1.0f + 0.5f * gamma * nrm;
#pragma unroll
    for (int c = 0; c < KS; ++c)
      if (4 * c + g == n) B[b][c] = cq;
  }
  float fpart[QB];
#pragma unroll
  for (int b = 0; b < QB; ++b) fpart[b] = 0.f;
  // Software pipeline: the MFMAs of tile t + 1 are issued before the vector
  // work on tile t's results, so that work does not wait on the matrix
  // unit's latency. The last iteration recomputes the last tile (in range,
  // results unused) instead of branching.
  auto contract = [&](int64_t t, rf4 (&d)[QB], rf4& W) {
    const float* T = tiles + t * rbf_tile_floats(KS);
    float Av[KS];
#pragma unroll
    for (int c = 0; c < KS; ++c) Av[c] = T[c * 64 + lane];
    const rf4 Cv = *reinterpret_cast<const rf4*>(T + 64 * KS + 4 * g);
    W = *reinterpret_cast<const rf4*>(T + 64 * KS + 16 + 4 * g);
#pragma unroll
    for (int b = 0; b < QB; ++b) {
      rf4 x = Cv;
#pragma unroll
      for (int c = 0; c < KS; ++c) x = __builtin_amdgcn_mfma_f32_16x16x4f32(Av[c], B[b][c], x, 0, 0, 0);
      d[b] = x;
    }
  };
  rf4 dcur[QB], Wcur;
  contract(0, dcur, Wcur);
  for (int64_t t = 0; t < ntiles; ++t) {
    rf4 dnxt[QB], Wnxt;
    contract(t + 1 < ntiles ? t + 1 : t, dnxt, Wnxt);
#pragma unroll
    for (int b = 0; b < QB; ++b) {
      float acc = fpart[b];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const float x = rbf_rcp_sat(dcur[b][r]);
        acc = fmaf(Wcur[r], x * x, acc);
      }
      fpart[b] = acc;
    }
#pragma unroll
    for (int b = 0; b < QB; ++b) dcur[b] = dnxt[b];
    Wcur = Wnxt;
  }
#pragma unroll
  for (int b = 0; b < QB; ++b) {
    float v = fpart[b];
    v += __shfl_xor(v, 16);
    v += __shfl_xor(v, 32);
    const int64_t j = qbase + 16 * b + col;
    if (g == 0 && j < N) {
      if (f) f[j] = v;
      if (label) label[j] = (v >= 0.0f) ? (int8_t)1 : (int8_t)-1;
    }
  }
}

__global__ void __launch_bounds__(256) k_rbf_empty(int64_t N, float* __restrict__ f, int8_t* __restrict__ label) {
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (j < N) {
    if (f) f[j] = 0.f;
    if (label) label[j] = 1;
  }
}

}  // namespace fastron

using namespace fastron;

extern "C" {

fastron_status fastron_rbf_score(const float* support_x, const float* alpha, int64_t S, int32_t n, float gamma,
                                 const float* q, int64_t N, float* f, int8_t* label, void* stream) {
  clear_error();
  FASTRON_CHECK(n >= 1 && n <= FASTRON_MAX_JOINTS, "n = %d outside [1, %d]", n, FASTRON_MAX_JOINTS);
  FASTRON_CHECK(S >= 0, "S = %lld < 0", (long long)S);
  FASTRON_CHECK(S == 0 || (support_x && alpha), "support_x and alpha must be non-NULL when S > 0");
  FASTRON_CHECK(std::isfinite(gamma) && gamma > 0.f, "gamma must be finite and > 0");
  FASTRON_CHECK(N >= 0, "N = %lld < 0", (long long)N);
  FASTRON_CHECK(N == 0 || q != nullptr, "q is NULL");
  FASTRON_CHECK(N == 0 || f != nullptr || label != nullptr, "f and label are both NULL");
  if (N == 0) return FASTRON_OK;
  hipStream_t s = as_stream(stream);
  const int64_t qblocks = (N + 255) / 256;
  FASTRON_CHECK(grid_fits(qblocks, 256), "N = %lld above one launch's 2^32 - 256 queries", (long long)N);
  if (S == 0) {
    hipLaunchKernelGGL(k_rbf_empty, dim3((unsigned)qblocks), dim3(256), 0, s, N, f, label);
    FASTRON_HIP(hipGetLastError());
    return FASTRON_OK;
  }
  const int KS = (n + 1 + 3) / 4;
  const int64_t ntiles = (S + 15) / 16;
  float* tiles = nullptr;
  FASTRON_HIP(hipMallocAsync(reinterpret_cast<void**>(&tiles), (size_t)ntiles * rbf_tile_floats(KS) * sizeof(float),
                             s));
  hipLaunchKernelGGL(k_rbf_prep, dim3((unsigned)((ntiles * 16 + 255) / 256)), dim3(256), 0, s, support_x, alpha, S,
                     (int)n, KS, ntiles, gamma, tiles);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) {
    const dim3 grid((unsigned)qblocks);
    switch (KS) {
      case 1: hipLaunchKernelGGL(k_score_rbf<1>, grid, dim3(256), 0, s, q, N, (int)n, gamma, tiles, ntiles, f, label); break;
      case 2: hipLaunchKernelGGL(k_score_rbf<2>, grid, dim3(256), 0, s, q, N, (int)n, gamma, tiles, ntiles, f, label); break;
      case 3: hipLaunchKernelGGL(k_score_rbf<3>, grid, dim3(256), 0, s, q, N, (int)n, gamma, tiles, ntiles, f, label); break;
      case 4: hipLaunchKernelGGL(k_score_rbf<4>, grid, dim3(256), 0, s, q, N, (int)n, gamma, tiles, ntiles, f, label); break;
      default: hipLaunchKernelGGL(k_score_rbf<5>, grid, dim3(256), 0, s, q, N, (int)n, gamma, tiles, ntiles, f, label); break;
    }
    e = hipGetLastError();
  }
  const hipError_t ef = hipFreeAsync(tiles, s);
  if (e == hipSuccess) e = ef;
  if (e != hipSuccess) return fail(FASTRON_EHIP, "configuration-space score launch failed: %s", hipGetErrorString(e));
  return FASTRON_OK;
}

}  // extern "C"

