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
// Each lane then sums 1/t^2 over m for its 4 (s, q) pairs, either with one
// saturated reciprocal and one FMA per value or, where the chain's reach
// bound allows it, as one running fraction with a single reciprocal per pair
// (wave_score_fp32); alpha_s / M weights the sum once per (s, q) and the four
// lane groups are reduced with shuffles at the end. Points fixed to the base contribute exactly 1 per pair and arrive as
// the constant f_const.
#include <cmath>
#include <mutex>

#include "score_device.h"

namespace fastron {

// ---------------------------------------------------------------------------
// FP32 MFMA form (default): one wave per 32 queries (two blocks of 16); the
// workgroup's 128 queries are staged (fused FK) by its first two waves, one
// query per lane. With two blocks the kernel fits 96 VGPRs for up to 8
// moving points, so 5 waves share a SIMD, and the finer workgroups leave a
// smaller partial last round. Four blocks per wave measured 3.7 % slower at
// S = 4,000, N = 1,000,000 and the same at 16,384 supports.
// ---------------------------------------------------------------------------
constexpr int kScoreBlocks = 2;
constexpr int kScoreQueriesPerBlock = kWavesPerBlock * 16 * kScoreBlocks;

// 5 waves per SIMD (96 VGPRs) up to 8 moving points; with the FP32 chain (fewer than 7 joints) 8 points need
// more registers, so 4 there
template <int MM, typename R, bool RAT>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(MM < 8 || sizeof(R) == 8 ? (MM <= 8 ? 5 : 1)
                                                                                                     : (MM <= 8 ? 4 : 1))))
k_score_mfma(ChainArgs c, const float* __restrict__ q, int64_t N, const char* __restrict__ blob, int64_t ntiles,
             int Mp, float gamma, float* __restrict__ f, int8_t* __restrict__ label) {
  static_assert(kScoreQueriesPerBlock % 64 == 0, "whole waves stage the workgroup's queries");
  __shared__ f4 lds[kScoreQueriesPerBlock][MM];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t bbase = (int64_t)blockIdx.x * kScoreQueriesPerBlock;
  if (wave < kScoreQueriesPerBlock / 64) stage_queries<MM, R>(c, q, N, gamma, bbase + 64 * wave + lane, lds + 64 * wave);
  __syncthreads();
  const float f_const = reinterpret_cast<const float*>(blob)[0];
  const float* tiles = reinterpret_cast<const float*>(blob + kHeaderBytes);
  const int wq = 16 * kScoreBlocks;
  wave_score_fp32<MM, kScoreBlocks, RAT, true>(lds + wq * wave, tiles, ntiles, Mp, f_const, bbase + wq * wave, N, f,
                                               label);
}

// ---------------------------------------------------------------------------
// VALU form: one query per lane, the cross term as three FMAs and an add
// against wave-uniform support operands (scalar loads), the per-pair sum in
// the same two forms as the MFMA kernels. Same result to FP32 rounding, no
// MFMA; kept as the baseline that the MFMA forms are measured against.
// ---------------------------------------------------------------------------
template <int MM, typename R, bool RAT>
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
    float n = RAT ? 1.f : 0.f, e = 0.f;
#pragma unroll
    for (int m = 0; m < MM; ++m) {
      const f4 v = V[s * Mp + m];
      const float t = fmaf(v[0], P[m][0], fmaf(v[1], P[m][1], fmaf(v[2], P[m][2], P[m][3] + v[3])));
      if constexpr (RAT) {
        const float tt = t * t;
        if (m == 0) {
          e = tt;
        } else {
          n = fmaf(n, tt, e);
          e *= tt;
        }
      } else {
        const float r = rcp_sat(t);
        n = fmaf(r, r, n);
      }
    }
    if constexpr (RAT) n *= __builtin_amdgcn_rcpf(e);
    acc_f = fmaf(w, n, acc_f);
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
// `grid` covers 256 queries per workgroup (VALU form); the MFMA form's
// workgroups take kScoreQueriesPerBlock.
template <int MM, typename R>
static void launch_one(uint32_t kind, bool rat, dim3 grid, hipStream_t s, const ChainArgs& c, const float* q,
                       int64_t N, const char* blob, int64_t nt, int Mp, float gamma, float* f, int8_t* label) {
  const dim3 gm((unsigned)((N + kScoreQueriesPerBlock - 1) / kScoreQueriesPerBlock));
  if (kind == FASTRON_SCORE_VALU && rat)
    hipLaunchKernelGGL((k_score_valu<MM, R, true>), grid, dim3(256), 0, s, c, q, N, blob, nt, Mp, gamma, f, label);
  else if (kind == FASTRON_SCORE_VALU)
    hipLaunchKernelGGL((k_score_valu<MM, R, false>), grid, dim3(256), 0, s, c, q, N, blob, nt, Mp, gamma, f, label);
  else if (rat)
    hipLaunchKernelGGL((k_score_mfma<MM, R, true>), gm, dim3(256), 0, s, c, q, N, blob, nt, Mp, gamma, f, label);
  else
    hipLaunchKernelGGL((k_score_mfma<MM, R, false>), gm, dim3(256), 0, s, c, q, N, blob, nt, Mp, gamma, f, label);
}

template <typename R>
static void launch_mm(int Mm, uint32_t kind, bool rat, dim3 grid, hipStream_t s, const ChainArgs& c, const float* q,
                      int64_t N, const char* blob, int64_t nt, int Mp, float gamma, float* f, int8_t* label) {
#define FASTRON_MM_CASE(K) \
  case K: launch_one<K, R>(kind, rat, grid, s, c, q, N, blob, nt, Mp, gamma, f, label); break;
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
  // the MFMA form's grid is the largest: two work-items per query
  FASTRON_CHECK(grid_fits((N + kScoreQueriesPerBlock - 1) / kScoreQueriesPerBlock, 256),
                "N = %lld above one launch's 2^31 - 128 queries", (long long)N);
  const char* blob = static_cast<const char*>(model->data);
  if (c.Mm == 0) {
    hipLaunchKernelGGL(k_score_const, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s, blob, N, f, label);
  } else {
    const bool rat = rational_sum_ok(c, model->gamma, kind == FASTRON_SCORE_BF16 && variant == 0 ? 256.0 : 65536.0);
    if (kind == FASTRON_SCORE_BF16)
      launch_score_bf16(c, variant, rat, dim3((unsigned)blocks), s, q, N, blob, nt, Mp, model->gamma, f, label);
    else if (c.n >= kFp64Joints)
      launch_mm<double>(c.Mm, kind, rat, dim3((unsigned)blocks), s, c, q, N, blob, nt, Mp, model->gamma, f, label);
    else
      launch_mm<float>(c.Mm, kind, rat, dim3((unsigned)blocks), s, c, q, N, blob, nt, Mp, model->gamma, f, label);
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
  FASTRON_CHECK(fastron::grid_fits((N + fastron::kScoreQueriesPerBlock - 1) / fastron::kScoreQueriesPerBlock, 256),
                "N = %lld above one launch's 2^31 - 128 queries", (long long)N);
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

int32_t fastron_score_rational(const fastron_chain* chain, const fastron_cpoints* cp, float gamma, uint32_t flags) {
  clear_error();
  ChainArgs c;
  fastron_status st = pack_chain(chain, cp, &c, true);
  if (st != FASTRON_OK) return st;
  FASTRON_CHECK(std::isfinite(gamma) && gamma > 0.f, "gamma must be finite and > 0");
  FASTRON_CHECK((flags & ~0x33u) == 0 && (flags & 3u) != 3u, "unknown flags 0x%x", flags);
  FASTRON_CHECK(((flags >> 4) & 3u) <= 2u, "unknown BF16 variant");
  const uint32_t kind = flags & 3u;
  const bool plain = kind == FASTRON_SCORE_BF16 && ((flags >> 4) & 3u) == 0u;
  return rational_sum_ok(c, gamma, plain ? 256.0 : 65536.0) ? 1 : 0;
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

// Scoring without allocation: the prepared support set goes into this
// file-scope device buffer (one copy per device, alive until the process
// ends) instead of stream-ordered scratch. Host code never passes the
// symbol itself to a kernel: its device address is looked up once per device
// with hipGetSymbolAddress and kept in g_noalloc_ptr.
static __device__ __align__(256) unsigned char scratch[FASTRON_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_noalloc_mu;
void* g_noalloc_ptr[kMaxDevices] = {};

fastron_status noalloc_scratch(void** out) {
  int dev = 0;
  FASTRON_HIP(hipGetDevice(&dev));
  FASTRON_CHECK(dev >= 0 && dev < kMaxDevices, "device %d outside [0, %d)", dev, kMaxDevices);
  std::lock_guard<std::mutex> lk(g_noalloc_mu);
  if (g_noalloc_ptr[dev] == nullptr) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || p == nullptr)
      return fail(FASTRON_EHIP, "hipGetSymbolAddress(scratch) failed on device %d: %s", dev, hipGetErrorString(e));
    g_noalloc_ptr[dev] = p;
  }
  *out = g_noalloc_ptr[dev];
  return FASTRON_OK;
}
}  // namespace

fastron_status fastron_fk_score_noalloc(const fastron_chain* chain, const fastron_cpoints* cp, const float* support_q,
                                        const float* alpha, int64_t S, float gamma, const float* q, int64_t N, float* f,
                                        int8_t* label, uint32_t flags, void* stream) {
  clear_error();
  ChainArgs c;
  fastron_status st = pack_chain(chain, cp, &c, true);
  if (st != FASTRON_OK) return st;
  FASTRON_CHECK(S >= 0, "S = %lld < 0", (long long)S);
  FASTRON_CHECK(S == 0 || (support_q && alpha), "support_q and alpha must be non-NULL when S > 0");
  FASTRON_CHECK(std::isfinite(gamma) && gamma > 0.f, "gamma must be finite and > 0");
  const int64_t bytes = fastron::model_bytes(S, c.M);
  FASTRON_CHECK(bytes <= FASTRON_NOALLOC_SCRATCH_BYTES,
                "S = %lld supports at M = %d need %lld bytes of prepared model; the static buffer holds %lld",
                (long long)S, c.M, (long long)bytes, (long long)FASTRON_NOALLOC_SCRATCH_BYTES);
  fastron_model probe{S, c.M, gamma, reinterpret_cast<void*>(256), bytes};
  st = check_score_args(c, &probe, q, N, f, label, flags);
  if (st != FASTRON_OK) return st;
  if (N == 0) return FASTRON_OK;
  void* blob = nullptr;
  st = noalloc_scratch(&blob);
  if (st != FASTRON_OK) return st;
  // fastron_support_prep writes every byte of the blob that the scoring kernels
  // read (header, every tile including padded supports), so nothing left by a
  // previous call survives into this one.
  fastron_model model{S, c.M, gamma, blob, bytes};
  st = fastron_support_prep(chain, cp, support_q, alpha, S, gamma, &model, stream);
  if (st != FASTRON_OK) return st;
  return score_launch(c, &model, q, N, f, label, flags, as_stream(stream));
}

}  // extern "C"
