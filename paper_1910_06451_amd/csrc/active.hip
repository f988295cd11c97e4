// Two-stage active learning of Section III-B (after each model update):
// assembly of the next update's training set on the device.
#include "fastron_internal.h"

// ---------------------------------------------------------------------------
// The training set of the next update is the support set, samples near each
// support point and uniform samples over the C-space. One thread per output
// row: rows [0, S) copy the supports (weights kept), rows S + s k + j are
// support s plus noise row s k + j (exploitation), and the last E rows copy
// the exploration samples; new rows get weight 0. The random draws are the
// caller's (noise and explore).
// ---------------------------------------------------------------------------
namespace fastron {
__global__ void __launch_bounds__(256) k_active_samples(const float* __restrict__ sq, const float* __restrict__ alpha,
                                                         int64_t S, int n, const float* __restrict__ noise, int k,
                                                         const float* __restrict__ explore, int64_t E,
                                                         float* __restrict__ X, float* __restrict__ alpha_out) {
  const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t nk = S * (int64_t)k;
  if (r >= S + nk + E) return;
  if (r < S) {
    for (int i = 0; i < n; ++i) X[r * n + i] = sq[r * n + i];
    if (alpha_out) alpha_out[r] = alpha[r];
  } else if (r < S + nk) {
    const int64_t e = r - S, s = e / k;
    for (int i = 0; i < n; ++i) X[r * n + i] = sq[s * n + i] + noise[e * n + i];
    if (alpha_out) alpha_out[r] = 0.f;
  } else {
    const int64_t e = r - S - nk;
    for (int i = 0; i < n; ++i) X[r * n + i] = explore[e * n + i];
    if (alpha_out) alpha_out[r] = 0.f;
  }
}

// Supports whose new label disagrees with the sign of their weight: weight 0.
__global__ void __launch_bounds__(256) k_active_relabel(const int8_t* __restrict__ y, int64_t S,
                                                         float* __restrict__ alpha) {
  const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (r >= S) return;
  const float a = alpha[r];
  if ((y[r] > 0 && a < 0.f) || (y[r] < 0 && a > 0.f)) alpha[r] = 0.f;
}
}  // namespace fastron

using namespace fastron;

extern "C" fastron_status fastron_active_samples(const float* support_q, const float* alpha, int64_t S, int32_t n,
                                                 const float* noise, int32_t k, const float* explore, int64_t E,
                                                 float* X_out, float* alpha_out, void* stream) {
  clear_error();
  FASTRON_CHECK(n >= 1 && n <= FASTRON_MAX_JOINTS, "n = %d outside [1, %d]", n, FASTRON_MAX_JOINTS);
  FASTRON_CHECK(S >= 0 && E >= 0 && k >= 0, "S, k and E must be >= 0");
  FASTRON_CHECK(S == 0 || support_q, "support_q is NULL");
  FASTRON_CHECK(S == 0 || k == 0 || noise, "noise is NULL");
  FASTRON_CHECK(E == 0 || explore, "explore is NULL");
  FASTRON_CHECK(alpha_out == nullptr || S == 0 || alpha, "alpha is NULL");
  const int64_t rows = S + S * (int64_t)k + E;
  if (rows == 0) return FASTRON_OK;
  FASTRON_CHECK(X_out != nullptr, "X_out is NULL");
  const int64_t blocks = (rows + 255) / 256;
  FASTRON_CHECK(grid_fits(blocks, 256), "%lld rows above one launch's 2^32 - 256", (long long)rows);
  hipLaunchKernelGGL(k_active_samples, dim3((unsigned)blocks), dim3(256), 0, as_stream(stream), support_q, alpha, S,
                     (int)n, noise, (int)k, explore, E, X_out, alpha_out);
  FASTRON_HIP(hipGetLastError());
  return FASTRON_OK;
}

extern "C" fastron_status fastron_active_relabel(const int8_t* y, int64_t S, float* alpha, void* stream) {
  clear_error();
  FASTRON_CHECK(S >= 0, "S < 0");
  if (S == 0) return FASTRON_OK;
  FASTRON_CHECK(y && alpha, "y and alpha must be non-NULL");
  const int64_t blocks = (S + 255) / 256;
  FASTRON_CHECK(grid_fits(blocks, 256), "S = %lld above one launch's 2^32 - 256", (long long)S);
  hipLaunchKernelGGL(k_active_relabel, dim3((unsigned)blocks), dim3(256), 0, as_stream(stream), y, S, alpha);
  FASTRON_HIP(hipGetLastError());
  return FASTRON_OK;
}
