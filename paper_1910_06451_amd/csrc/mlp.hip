// Learned screening: a small MLP on the FK control points (3M inputs ->
// H -> H -> 1 logit, ReLU), trained with BCE-with-logits and Adam, run as a
// pre-screen whose uncertain queries (|logit| < tau) fall back to the Fastron
// FK score. Not part of the paper's method; the paper cites a network on
// control points (for self-collision cost) as prior art.
//
// Precision: BF16 operands on the matrix cores (v_mfma_f32_16x16x32_bf16)
// with FP32 accumulation; FP32 master weights, biases, pre-activations,
// head, loss and optimiser state.
//
// Kernels:
//   k_gemm_bf16      C = act(A B + bias), A / B bf16 with arbitrary strides
//                    (so transposes are free), 64 x 64 output tile per
//                    workgroup, K staged through LDS in chunks of 32; the
//                    epilogue can write FP32 and/or BF16, or reduce the row
//                    against the head weights (fused last layer).
//   k_mlp_input      gathers / computes FK features and standardises them
//   k_colsum         deterministic two-pass column sums (bias gradients)
//   k_head_*         logit, loss and dlogit; last-layer gradients
//   k_adam           Adam on the FP32 masters + BF16 copies
#include <cmath>
#include <cstring>
#include <vector>

#include "fastron_internal.h"

struct fastron_mlp;

namespace fastron {

typedef float f4m __attribute__((ext_vector_type(4)));
typedef __bf16 bf8m __attribute__((ext_vector_type(8)));
typedef unsigned short u8m __attribute__((ext_vector_type(8)));

typedef float f2m __attribute__((ext_vector_type(2)));
typedef __bf16 b2m __attribute__((ext_vector_type(2)));
typedef short s2m __attribute__((ext_vector_type(2)));
typedef unsigned u4m __attribute__((ext_vector_type(4)));

// FP32 -> BF16, round to nearest even (the hardware conversion).
__device__ __forceinline__ uint16_t to_bf16(float x) {
  const b2m h = __builtin_convertvector((f2m){x, 0.f}, b2m);
  return (uint16_t)__builtin_bit_cast(uint32_t, h);
}
// Two FP32 values -> packed BF16 pair (RNE) with ReLU applied on the BF16 bit
// patterns: a BF16 value is negative exactly when its bits, read as int16,
// are negative, so an int16 max with 0 is the ReLU.
__device__ __forceinline__ uint32_t relu_bf16x2(float a, float b) {
  const b2m h = __builtin_convertvector((f2m){a, b}, b2m);
  return __builtin_bit_cast(uint32_t, __builtin_elementwise_max(__builtin_bit_cast(s2m, h), (s2m){0, 0}));
}
__device__ __forceinline__ float from_bf16(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// ---------------------------------------------------------------------------
// Generic BF16 GEMM
// ---------------------------------------------------------------------------
struct GemmArgs {
  const uint16_t* A;
  int64_t sam, sak;  // A(m, k) = A[m * sam + k * sak]
  const uint16_t* B;
  int64_t sbk, sbn;  // B(k, n) = B[k * sbk + n * sbn]
  float* C;          // optional FP32 output C[m * ldc + n]
  int64_t ldc;
  uint16_t* Cb;      // optional BF16 output Cb[m * ldcb + n]
  int64_t ldcb;
  const float* bias; // optional [N]
  const float* head; // optional [N]: fused last layer, partial[n_tile][m] = sum_n act(..) * head[n]
  float* partial;    // [ceil(N / 64)][M] when head is set
  int relu;
  int M, N, K;
  int kchunk;        // K range per blockIdx.z (a multiple of the K chunk)
  float* split;      // split-K: raw partial products [gridDim.z][M][N], no epilogue
};

constexpr int kGT = 64;   // output tile edge
constexpr int kGK = 32;   // K chunk
constexpr int kGPad = 8;  // LDS row padding (elements)

__global__ void __launch_bounds__(256) k_gemm_bf16(GemmArgs g) {
  __shared__ __align__(16) uint16_t As[kGT][kGK + kGPad];
  __shared__ __align__(16) uint16_t Bs[kGT][kGK + kGPad];  // stored transposed: Bs[n][k]
  __shared__ float hsum[4][kGT];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t m0 = (int64_t)blockIdx.x * kGT, n0 = (int64_t)blockIdx.y * kGT;
  const int64_t kb = (int64_t)blockIdx.z * g.kchunk;
  const int64_t ke = kb + g.kchunk < g.K ? kb + g.kchunk : g.K;
  f4m acc[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) acc[t] = (f4m){0.f, 0.f, 0.f, 0.f};
  for (int64_t k0 = kb; k0 < ke; k0 += kGK) {
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int e = tid * 8 + i;  // 2048 elements per operand chunk
      const int r = e / kGK, kk = e % kGK;
      const int64_t gm = m0 + r, gk = k0 + kk, gn = n0 + r;
      As[r][kk] = (gm < g.M && gk < ke) ? g.A[gm * g.sam + gk * g.sak] : (uint16_t)0;
      Bs[r][kk] = (gn < g.N && gk < ke) ? g.B[gk * g.sbk + gn * g.sbn] : (uint16_t)0;
    }
    __syncthreads();
    const int row = 16 * wave + (lane & 15), kq = 8 * (lane >> 4);
    const bf8m a = __builtin_bit_cast(bf8m, *reinterpret_cast<const u8m*>(&As[row][kq]));
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const bf8m b = __builtin_bit_cast(bf8m, *reinterpret_cast<const u8m*>(&Bs[16 * t + (lane & 15)][kq]));
      acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[t], 0, 0, 0);
    }
    __syncthreads();
  }
  // epilogue: lane holds rows 16 wave + 4 (lane / 16) + r, column 16 t + lane % 16
  if (g.split) {
    float* out = g.split + (int64_t)blockIdx.z * g.M * g.N;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int64_t n = n0 + 16 * t + (lane & 15);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t m = m0 + 16 * wave + 4 * (lane >> 4) + r;
        if (m < g.M && n < g.N) out[m * g.N + n] = acc[t][r];
      }
    }
    return;
  }
  float hpart[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int64_t n = n0 + 16 * t + (lane & 15);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t m = m0 + 16 * wave + 4 * (lane >> 4) + r;
      if (m < g.M && n < g.N) {
        float v = acc[t][r];
        if (g.bias) v += g.bias[n];
        if (g.relu) v = fmaxf(v, 0.f);
        if (g.C) g.C[m * g.ldc + n] = v;
        if (g.Cb) g.Cb[m * g.ldcb + n] = to_bf16(v);
        if (g.head) hpart[r] += v * g.head[n];
      }
    }
  }
  if (g.head) {
    // reduce the 64 columns of this tile for each row: lanes sharing lane / 16 hold the same rows
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      float v = hpart[r];
      v += __shfl_xor(v, 1);
      v += __shfl_xor(v, 2);
      v += __shfl_xor(v, 4);
      v += __shfl_xor(v, 8);
      if ((lane & 15) == 0) hsum[wave][4 * (lane >> 4) + r] = v;
    }
    __syncthreads();
    if (tid < kGT) {
      const int w = tid >> 4, rr = tid & 15;
      const int64_t m = m0 + 16 * w + rr;
      if (m < g.M) g.partial[(int64_t)blockIdx.y * g.M + m] = hsum[w][rr];
    }
  }
}

// Split-K: sums the partial products in split order (deterministic) and
// applies the epilogue (bias, ReLU, FP32 / BF16 output).
__global__ void __launch_bounds__(256) k_splitk_reduce(const float* __restrict__ split, int splits, int M, int N,
                                                        const float* __restrict__ bias, int relu,
                                                        float* __restrict__ C, int64_t ldc, uint16_t* __restrict__ Cb,
                                                        int64_t ldcb) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t MN = (int64_t)M * N;
  if (e >= MN) return;
  const int64_t m = e / N, n = e % N;
  float v = 0.f;
  for (int z = 0; z < splits; ++z) v += split[z * MN + e];
  if (bias) v += bias[n];
  if (relu) v = fmaxf(v, 0.f);
  if (C) C[m * ldc + n] = v;
  if (Cb) Cb[m * ldcb + n] = to_bf16(v);
}

// ---------------------------------------------------------------------------
// Inputs: standardised control points as BF16 rows of width kin_pad
// ---------------------------------------------------------------------------
// From stored control points P [N][M][3], rows selected by `order` (or identity).
// An index outside [0, n_rows) is not followed: the row reads as zeros and
// *bad is set (the caller reports FASTRON_EINVAL).
__global__ void __launch_bounds__(256) k_mlp_input_points(const float* __restrict__ P, const int32_t* __restrict__ order,
                                                           int64_t row0, int64_t rows, int64_t n_rows, int d_in,
                                                           int kin_pad, const float* __restrict__ mu,
                                                           const float* __restrict__ sd, uint16_t* __restrict__ X,
                                                           float* __restrict__ Xf, int* __restrict__ bad) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= rows * kin_pad) return;
  const int64_t r = e / kin_pad;
  const int c = (int)(e % kin_pad);
  const int64_t src = order ? (int64_t)order[row0 + r] : row0 + r;
  const bool ok = src >= 0 && src < n_rows;
  if (!ok && c == 0) *bad = 1;
  const float v = (c < d_in && ok) ? (P[src * d_in + c] - mu[c]) / sd[c] : 0.f;
  X[e] = to_bf16(v);
  if (Xf) Xf[e] = v;
}

// From joint configurations: FK fused (one thread per query).
template <typename R>
__global__ void __launch_bounds__(256) k_mlp_input_fk(ChainArgs c, const float* __restrict__ q, int64_t row0,
                                                       int64_t rows, int kin_pad, const float* __restrict__ mu,
                                                       const float* __restrict__ sd, uint16_t* __restrict__ X) {
  const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (r >= rows) return;
  float qv[FASTRON_MAX_JOINTS];
  for (int i = 0; i < c.n; ++i) qv[i] = q[(row0 + r) * c.n + i];
  uint16_t* row = X + r * kin_pad;
  for (int k = 3 * c.M; k < kin_pad; ++k) row[k] = 0;
  fk_walk<R>(c, qv, [&](int m, float x, float y, float z) {
    row[3 * m + 0] = to_bf16((x - mu[3 * m + 0]) / sd[3 * m + 0]);
    row[3 * m + 1] = to_bf16((y - mu[3 * m + 1]) / sd[3 * m + 1]);
    row[3 * m + 2] = to_bf16((z - mu[3 * m + 2]) / sd[3 * m + 2]);
  });
}

// Feature statistics over N rows (one block per feature, fixed order): mean and
// standard deviation; a constant feature gets sd = 1.
__global__ void __launch_bounds__(256) k_feat_stats(const float* __restrict__ P, int64_t N, int d_in,
                                                     float* __restrict__ mu, float* __restrict__ sd) {
  __shared__ double part[256];
  const int c = blockIdx.x;
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < N; i += 256) s += (double)P[i * d_in + c];
  part[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
    __syncthreads();
  }
  const double mean = part[0] / (double)N;
  __syncthreads();
  double v = 0.0;
  for (int64_t i = threadIdx.x; i < N; i += 256) {
    const double d = (double)P[i * d_in + c] - mean;
    v += d * d;
  }
  part[threadIdx.x] = v;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double var = part[0] / (double)N;
    mu[c] = (float)mean;
    sd[c] = var > 1e-12 ? (float)sqrt(var) : 1.0f;
  }
}

// ---------------------------------------------------------------------------
// Head: z = sum of the fused partials + b3; BCE loss and dz = (sigmoid(z) - t) / B
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_head_forward(const float* __restrict__ partial, int ntiles, int64_t rows,
                                                       const float* __restrict__ b3, float* __restrict__ z) {
  const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (r >= rows) return;
  float v = b3[0];
  for (int t = 0; t < ntiles; ++t) v += partial[(int64_t)t * rows + r];
  z[r] = v;
}

__global__ void __launch_bounds__(256) k_bce(const float* __restrict__ z, const int8_t* __restrict__ y,
                                              const int32_t* __restrict__ order, int64_t row0, int64_t rows,
                                              int64_t n_rows, float* __restrict__ dz, float* __restrict__ loss_part) {
  __shared__ float part[256];
  const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
  float l = 0.f;
  if (r < rows) {
    int64_t src = order ? (int64_t)order[row0 + r] : row0 + r;
    if (src < 0 || src >= n_rows) src = 0;  // flagged by the input kernel
    const float t = y[src] > 0 ? 1.f : 0.f;
    const float zz = z[r];
    l = fmaxf(zz, 0.f) + log1pf(expf(-fabsf(zz))) - t * zz;
    const float sig = 1.f / (1.f + expf(-zz));
    dz[r] = (sig - t) / (float)rows;
  }
  part[threadIdx.x] = l;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) loss_part[blockIdx.x] = part[0];
}

// dZ2 = dz w3 [Z2 > 0] (FP32 and BF16)
__global__ void __launch_bounds__(256) k_head_back(const float* __restrict__ dz, const float* __restrict__ w3,
                                                    const float* __restrict__ Z2, int64_t rows, int H,
                                                    float* __restrict__ dZ2, uint16_t* __restrict__ dZ2b) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= rows * H) return;
  const int64_t r = e / H;
  const int c = (int)(e % H);
  const float v = Z2[e] > 0.f ? dz[r] * w3[c] : 0.f;
  dZ2[e] = v;
  dZ2b[e] = to_bf16(v);
}

// dZ1 = dH1 [Z1 > 0]
__global__ void __launch_bounds__(256) k_relu_back(const float* __restrict__ dH, const float* __restrict__ Z,
                                                    int64_t n, float* __restrict__ dZ, uint16_t* __restrict__ dZb) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= n) return;
  const float v = Z[e] > 0.f ? dH[e] : 0.f;
  dZ[e] = v;
  dZb[e] = to_bf16(v);
}

// out[c] = sum_r X[r * ld + c] * (s ? s[r] : 1), two passes with a fixed order:
// pass 1 writes partials[chunk][c] for 64 row chunks, pass 2 sums them.
constexpr int kColChunks = 64;
__global__ void __launch_bounds__(256) k_colsum_pass1(const float* __restrict__ X, int64_t rows, int cols, int64_t ld,
                                                       const float* __restrict__ s, float* __restrict__ partials) {
  const int c = blockIdx.x * 256 + threadIdx.x;
  const int chunk = blockIdx.y;
  if (c >= cols) return;
  const int64_t per = (rows + kColChunks - 1) / kColChunks;
  const int64_t r0 = chunk * per, r1 = r0 + per < rows ? r0 + per : rows;
  float acc = 0.f;
  for (int64_t r = r0; r < r1; ++r) acc += X[r * ld + c] * (s ? s[r] : 1.f);
  partials[(int64_t)chunk * cols + c] = acc;
}
__global__ void __launch_bounds__(256) k_colsum_pass2(const float* __restrict__ partials, int cols,
                                                       float* __restrict__ out) {
  const int c = blockIdx.x * 256 + threadIdx.x;
  if (c >= cols) return;
  float acc = 0.f;
  for (int k = 0; k < kColChunks; ++k) acc += partials[(int64_t)k * cols + c];
  out[c] = acc;
}

// relu(Z2) . w  -> used for gw3 = sum_r relu(Z2[r]) dz[r]: relu applied on the fly
__global__ void __launch_bounds__(256) k_relu_copy(const float* __restrict__ Z, int64_t n, float* __restrict__ H) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e < n) H[e] = fmaxf(Z[e], 0.f);
}

// Adam (Kingma & Ba) on FP32 masters; c1 = 1 / (1 - beta1^t), c2 = 1 / (1 - beta2^t).
__global__ void __launch_bounds__(256) k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                                               float* __restrict__ v, int64_t n, float lr, float b1, float b2,
                                               float eps, float c1, float c2) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi * c1) / (sqrtf(vi * c2) + eps);
}

// BF16 copies of the weight matrices (W1 padded to kin_pad rows).
__global__ void __launch_bounds__(256) k_weights_bf16(const float* __restrict__ w1, const float* __restrict__ w2,
                                                       int d_in, int kin_pad, int H, uint16_t* __restrict__ w1b,
                                                       uint16_t* __restrict__ w2b) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t n1 = (int64_t)kin_pad * H, n2 = (int64_t)H * H;
  if (e < n1) {
    const int64_t r = e / H;
    w1b[e] = r < d_in ? to_bf16(w1[e]) : (uint16_t)0;
  } else if (e < n1 + n2) {
    w2b[e - n1] = to_bf16(w2[e - n1]);
  }
}

// Screening decision: confident logits give the label directly; the others are
// appended to the fallback list (order of appends is irrelevant: each query's
// result depends only on itself).
__global__ void __launch_bounds__(256) k_screen(const float* __restrict__ z, int64_t row0, int64_t rows, float tau,
                                                 float* __restrict__ logit_out, int8_t* __restrict__ label,
                                                 uint8_t* __restrict__ fell_back, int32_t* __restrict__ fb_idx,
                                                 unsigned long long* __restrict__ fb_count) {
  const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (r >= rows) return;
  const float v = z[r];
  const int64_t j = row0 + r;
  if (logit_out) logit_out[j] = v;
  const bool fb = fabsf(v) < tau;
  if (fell_back) fell_back[j] = fb ? 1 : 0;
  if (fb) {
    const unsigned long long k = atomicAdd(fb_count, 1ull);
    fb_idx[k] = (int32_t)j;
  } else {
    label[j] = v >= 0.f ? (int8_t)1 : (int8_t)-1;
  }
}

__global__ void __launch_bounds__(256) k_gather_rows(const float* __restrict__ q, int n, const int32_t* __restrict__ idx,
                                                      const unsigned long long* __restrict__ count,
                                                      float* __restrict__ out) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t cnt = (int64_t)*count;
  if (e >= cnt * n) return;
  const int64_t r = e / n;
  out[e] = q[(int64_t)idx[r] * n + (e % n)];
}

__global__ void __launch_bounds__(256) k_scatter_labels(const int8_t* __restrict__ lab_sub, const float* __restrict__ f_sub,
                                                         const int32_t* __restrict__ idx,
                                                         const unsigned long long* __restrict__ count,
                                                         int8_t* __restrict__ label, float* __restrict__ f_out) {
  const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (r >= (int64_t)*count) return;
  label[idx[r]] = lab_sub[r];
  if (f_out) f_out[idx[r]] = f_sub[r];
}

__global__ void k_zero_u64(unsigned long long* p) {
  if (threadIdx.x == 0) *p = 0ull;
}

// ---------------------------------------------------------------------------
// Fused screening inference for the 3M (<= 24) -> 256 -> 256 -> 1 network
// ---------------------------------------------------------------------------
// One persistent workgroup per CU holds W2 (BF16, 128 KB) in LDS for its whole
// life and walks tiles of 512 queries; each of its 8 waves owns 64 queries
// (four 16-query blocks). Per tile a wave
//   1. computes the FK of its 64 queries (one per lane, FP32 chain with
//      hardware sin / cos), standardises them and stages the BF16 features
//      in LDS;
//   2. layer 1 on the matrix cores in transposed form, H1^T = W1^T X^T, so
//      that every lane ends up holding exactly the H1 values it must feed to
//      layer 2 as an MFMA operand (no trip through LDS): the rows of each W1^T
//      fragment are permuted so that lane group g (lanes 16g..16g+15) receives
//      hidden units 32c + 8g .. 32c + 8g + 7 of chunk c;
//   3. layer 2 as H2^T = W2^T H1^T, each W2 fragment read from LDS once and
//      applied to the four query blocks, with bias, ReLU and the head
//      (dot with w3) in the epilogue;
//   4. reduces the head partials across lane groups, adds b3 and takes the
//      screening decision (one atomic per workgroup and tile reserves the
//      room for its fallback queries).
// The BF16 rounding points (X, H1) and the FP32 accumulation are those of the
// staged GEMM path; the biases enter as the accumulators' initial values
// instead of being added after the product (rounding differs in the last FP32
// place).
constexpr int kInfH = 256;    // hidden width served by the fused kernel
constexpr int kInfXRow = 24;  // staged features per query (input width <= 24, i.e. M <= 8)
constexpr int kInfWaves = 8;  // two waves per SIMD: one's VALU work overlaps the other's MFMAs
constexpr int kInfTile = 64 * kInfWaves;

// Layer-1 fragment v (0..15) covers hidden units 32 (v / 2) + 8 g + 4 (v % 2) + i at MFMA output
// row 4 g + i of the transposed product.
__device__ __host__ __forceinline__ int inf_unit1(int v, int row) {
  return 32 * (v >> 1) + 8 * (row >> 2) + 4 * (v & 1) + (row & 3);
}

// Packs the FP32 masters into MFMA operand order:
//   w1p[v][lane][j] = W1[8 (lane / 16) + j][inf_unit1(v, lane % 16)]   (zero past d_in)
//   w2p[nb][c][lane][j] = W2[32 c + 8 (lane / 16) + j][16 nb + lane % 16]
__global__ void __launch_bounds__(256) k_pack_infer(const float* __restrict__ w1, const float* __restrict__ w2,
                                                     const float* __restrict__ sd, int d_in,
                                                     uint16_t* __restrict__ w1p, uint16_t* __restrict__ w2p,
                                                     float* __restrict__ isd) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e < d_in) isd[e] = 1.0f / sd[e];
  constexpr int64_t n1 = 16 * 64 * 8, n2 = (int64_t)kInfH * kInfH;
  if (e < n1) {
    const int j = (int)(e & 7), lane = (int)((e >> 3) & 63), v = (int)(e >> 9);
    const int k = 8 * (lane >> 4) + j;
    w1p[e] = k < d_in ? to_bf16(w1[(int64_t)k * kInfH + inf_unit1(v, lane & 15)]) : (uint16_t)0;
  } else if (e < n1 + n2) {
    const int64_t f = e - n1;
    const int j = (int)(f & 7), lane = (int)((f >> 3) & 63), c = (int)((f >> 9) & 7), nb = (int)(f >> 12);
    const int k = 32 * c + 8 * (lane >> 4) + j;
    w2p[f] = to_bf16(w2[(int64_t)k * kInfH + 16 * nb + (lane & 15)]);
  }
}

struct InferArgs {
  ChainArgs c;
  const float* q;
  int64_t N;
  int64_t ntiles;
  const float* mu;
  const float* isd;  // 1 / sd
  const uint16_t* w1p;
  const float* b1;
  const uint16_t* w2p;
  const float* b2;
  const float* w3;
  const float* b3;
  float tau;
  float* logit;
  int8_t* label;
  uint8_t* fell_back;
  int32_t* fb_idx;
  unsigned long long* fb_count;
};

__global__ void __launch_bounds__(kInfTile) k_mlp_screen_fused(InferArgs a) {
  __shared__ __align__(16) uint16_t w2s[kInfH * kInfH];
  __shared__ __align__(16) uint16_t xs[kInfWaves][64][kInfXRow];
  __shared__ __align__(16) float b1s[kInfH], b2s[kInfH], w3s[kInfH];
  __shared__ unsigned fb_wave[kInfWaves];
  __shared__ unsigned long long fb_base;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, g = lane >> 4;
  {
    const u8m* src = reinterpret_cast<const u8m*>(a.w2p);
    u8m* dst = reinterpret_cast<u8m*>(w2s);
    for (int i = tid; i < kInfH * kInfH / 8; i += kInfTile) dst[i] = src[i];
    for (int i = tid; i < kInfH; i += kInfTile) {
      b1s[i] = a.b1[i];
      b2s[i] = a.b2[i];
      w3s[i] = a.w3[i];
    }
  }
  const float b3 = a.b3[0];
  uint16_t* xrow = &xs[wave][lane][0];
  for (int64_t tile = blockIdx.x; tile < a.ntiles; tile += gridDim.x) {
    __syncthreads();  // W2 staged (first tile); this wave's previous features consumed
    const int64_t qi = tile * kInfTile + 64 * wave + lane;
    // 1. FK + standardisation of this lane's query into its LDS row
#pragma unroll
    for (int t = 0; t < kInfXRow / 8; ++t) *reinterpret_cast<u8m*>(xrow + 8 * t) = (u8m){0, 0, 0, 0, 0, 0, 0, 0};
    if (qi < a.N) {
      float qv[FASTRON_MAX_JOINTS];
      for (int i = 0; i < a.c.n; ++i) qv[i] = a.q[qi * a.c.n + i];
      fk_walk<FastTrig>(a.c, qv, [&](int m, float x, float y, float z) {
        xrow[3 * m + 0] = to_bf16((x - a.mu[3 * m + 0]) * a.isd[3 * m + 0]);
        xrow[3 * m + 1] = to_bf16((y - a.mu[3 * m + 1]) * a.isd[3 * m + 1]);
        xrow[3 * m + 2] = to_bf16((z - a.mu[3 * m + 2]) * a.isd[3 * m + 2]);
      });
    }
    __syncthreads();
    // 2. layer 1 (transposed): per fragment v, D[row = unit][col = query]
    // lane group g holds features 8g .. 8g + 7 (group 3: the zero padding 24 .. 31)
    bf8m xb[4];
#pragma unroll
    for (int qb = 0; qb < 4; ++qb)
      xb[qb] = g < 3 ? __builtin_bit_cast(bf8m, *reinterpret_cast<const u8m*>(&xs[wave][16 * qb + (lane & 15)][8 * g]))
                     : __builtin_bit_cast(bf8m, (u8m){0, 0, 0, 0, 0, 0, 0, 0});
    // the bias enters as the accumulator's initial value; ReLU and the BF16
    // rounding are applied to pairs of outputs
    u4m h1[4][8];
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const bf8m w = __builtin_bit_cast(bf8m, reinterpret_cast<const u8m*>(a.w1p)[v * 64 + lane]);
      const f4m bias = *reinterpret_cast<const f4m*>(&b1s[32 * (v >> 1) + 8 * g + 4 * (v & 1)]);
#pragma unroll
      for (int qb = 0; qb < 4; ++qb) {
        const f4m d = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w, xb[qb], bias, 0, 0, 0);
        h1[qb][v >> 1][2 * (v & 1)] = relu_bf16x2(d[0], d[1]);
        h1[qb][v >> 1][2 * (v & 1) + 1] = relu_bf16x2(d[2], d[3]);
      }
    }
    // 3. layer 2 (transposed): bias as the initial accumulator, ReLU and the
    //    head (dot with w3) in the epilogue
    float lp[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll 1
    for (int nb = 0; nb < kInfH / 16; ++nb) {
      const f4m bias = *reinterpret_cast<const f4m*>(&b2s[16 * nb + 4 * g]);
      f4m acc[4];
#pragma unroll
      for (int qb = 0; qb < 4; ++qb) acc[qb] = bias;
#pragma unroll
      for (int c = 0; c < 8; ++c) {
        const bf8m w = __builtin_bit_cast(bf8m, reinterpret_cast<const u8m*>(w2s)[(nb * 8 + c) * 64 + lane]);
#pragma unroll
        for (int qb = 0; qb < 4; ++qb)
          acc[qb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w, __builtin_bit_cast(bf8m, h1[qb][c]), acc[qb], 0, 0, 0);
      }
      const f4m head = *reinterpret_cast<const f4m*>(&w3s[16 * nb + 4 * g]);
#pragma unroll
      for (int qb = 0; qb < 4; ++qb)
#pragma unroll
        for (int i = 0; i < 4; ++i) lp[qb] = fmaf(fmaxf(acc[qb][i], 0.f), head[i], lp[qb]);
    }
    // 4. head: sum the four lane groups; lane l then owns query 64 wave + l
#pragma unroll
    for (int qb = 0; qb < 4; ++qb) {
      lp[qb] += __shfl_xor(lp[qb], 16);
      lp[qb] += __shfl_xor(lp[qb], 32);
    }
    const float z = (g == 0 ? lp[0] : g == 1 ? lp[1] : g == 2 ? lp[2] : lp[3]) + b3;
    const bool valid = qi < a.N;
    const bool fb = valid && fabsf(z) < a.tau;
    if (valid) {
      if (a.logit) a.logit[qi] = z;
      if (a.fell_back) a.fell_back[qi] = fb ? 1 : 0;
      if (!fb) a.label[qi] = z >= 0.f ? (int8_t)1 : (int8_t)-1;
    }
    // fallback list: one atomic per workgroup and tile, then each wave writes
    // its queries behind those of the lower waves
    const unsigned long long ballot = __ballot(fb);
    if (lane == 0) fb_wave[wave] = (unsigned)__popcll(ballot);
    __syncthreads();
    if (tid == 0) {
      unsigned tot = 0;
      for (int w = 0; w < kInfWaves; ++w) tot += fb_wave[w];
      fb_base = tot ? atomicAdd(a.fb_count, (unsigned long long)tot) : 0ull;
    }
    __syncthreads();
    if (fb) {
      unsigned long long off = fb_base;
      for (int w = 0; w < wave; ++w) off += fb_wave[w];
      a.fb_idx[off + __popcll(ballot & ((1ull << lane) - 1ull))] = (int32_t)qi;
    }
  }
}

// ---------------------------------------------------------------------------
// Training step for the 3M (<= 32) -> 256 -> 256 -> 1 network: three kernels
// per batch instead of the staged GEMM sequence.
//   k_train_rows   per 16 batch rows, four waves that each own a quarter of
//                  the hidden units: standardised BF16 inputs, layer 1 (all
//                  units: the operand of layer 2) and layer 2 (own units) in
//                  transposed form (hidden units as MFMA rows, batch rows as
//                  columns, as in the screening kernel), the head's partial
//                  sums over own units (added in LDS in a fixed order), loss,
//                  dZ2 = [Z2 > 0] dz w3 (own units, shared through LDS), then
//                  dH1^T = W2 dZ2^T and dZ1 = [Z1 > 0] dH1 for own units;
//                  writes X, H1, dZ2 and dZ1 unit-major (each unit's batch
//                  rows contiguous) for the weight gradients, and
//                  per-workgroup sums over its rows for the bias and head
//                  gradients and the loss. Splitting the units fills the
//                  device with a batch of 8,192 rows: 256 workgroups of 8 waves
//                  (two 16-row blocks), all sharing one staged copy of the
//                  W2 operands, instead of one wave per 16 rows.
//   k_train_wgrad  gW2 = H1^T dZ2 and gW1 = X^T dZ1, contracting over the
//                  batch rows in split-K slices (one partial per slice).
//   k_train_adam   sums the partials in a fixed order, applies Adam to the
//                  FP32 masters and refreshes every BF16 operand copy.
// Layer 2 permutes its output units like layer 1 (fragment v, row 4 g + i is
// unit inf_unit1(v, 4 g + i)), so that lane group g holds units
// 32 c + 8 g .. + 7 of chunk c: exactly the operand dH1^T = W2 dZ2^T needs,
// and the order in which dH1^T comes out is that of H1 (whose nonzero entries
// are the ReLU mask). Rounding points are those of the staged path: X, W1,
// H1, W2, dZ2 and dZ1 in BF16, everything else FP32.
// ---------------------------------------------------------------------------
constexpr int kTrH = 256;        // hidden width of the training kernels
constexpr int kTrIn = 32;        // input features, zero-padded
constexpr int kTrBlocks = 2;     // 16-row blocks per workgroup of k_train_rows
constexpr int kTrSlices = 4;     // hidden-unit slices per block (one wave each)
constexpr int kTrWaves = kTrBlocks * kTrSlices;
constexpr int kTrThreads = 64 * kTrWaves;
constexpr int kTrRows = 16 * kTrBlocks;
constexpr int kTrSliceV = 16 / kTrSlices;  // layer fragments (16 units each) per slice
constexpr int kTrSliceC = 8 / kTrSlices;   // chunks of 32 units per slice
constexpr int kTrVec = 3 * kTrH + 2;  // per-workgroup sums: gb1, gb2, gw3, gb3, loss
constexpr int kTrSplitsMax = 32;      // split-K slices of the weight-gradient kernel

__device__ __forceinline__ uint32_t pack_bf16x2(float a, float b) {
  const b2m h = __builtin_convertvector((f2m){a, b}, b2m);
  return __builtin_bit_cast(uint32_t, h);
}
__device__ __forceinline__ uint16_t bf16_at(const u4m& v, int j) {
  return (uint16_t)((v[j >> 1] >> (16 * (j & 1))) & 0xffffu);
}
// Sum over the 16 batch rows of a wave (the 16 lanes of a row of the wave,
// lane / 16 equal, hold the same hidden units of different batch rows); every
// lane of the 16 gets it. Four DPP adds in a fixed order: quad_perm [1,0,3,2],
// quad_perm [2,3,0,1], row_half_mirror, row_mirror.
__device__ __forceinline__ float dpp_add(float v, int ctrl_sel) {
  int o;
  switch (ctrl_sel) {
    case 0: o = __builtin_amdgcn_update_dpp(0, __float_as_int(v), 0xB1, 0xF, 0xF, false); break;
    case 1: o = __builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x4E, 0xF, 0xF, false); break;
    case 2: o = __builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x141, 0xF, 0xF, false); break;
    default: o = __builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x140, 0xF, 0xF, false); break;
  }
  return v + __int_as_float(o);
}
__device__ __forceinline__ float rows_sum(float v) {
  v = dpp_add(v, 0);
  v = dpp_add(v, 1);
  v = dpp_add(v, 2);
  return dpp_add(v, 3);
}

// Writes a wave's 16 batch rows x 64 units (units 64 us .. + 63) of BF16
// values (lane (g, col) holding units 64 us + 32 cc + 8 g .. + 7 of row col in
// u4m v[cc]) unit-major to T[unit][row0 + row] through the wave's LDS area
// `st` ([unit][24] halfwords: 16 rows and a pad that spreads the four lane
// groups over the banks), so that each lane stores 16 bytes (8 rows of one
// unit) at a time.
constexpr int kTrStageStride = 24;
__device__ __forceinline__ void store_unit_major(const u4m* v, int us, uint16_t* st, uint16_t* __restrict__ T,
                                                 int64_t ldT, int64_t row0, int lane) {
  const int g = lane >> 4, col = lane & 15;
#pragma unroll
  for (int cc = 0; cc < kTrSliceC; ++cc)
#pragma unroll
    for (int j = 0; j < 8; ++j) st[(32 * cc + 8 * g + j) * kTrStageStride + col] = bf16_at(v[cc], j);
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  constexpr int kUnits = kTrH / kTrSlices;
#pragma unroll
  for (int q = 0; q < 2 * kUnits / 64; ++q) {
    const int chunk = q * 64 + lane;  // unit = chunk / 2 of the slice, rows 8 (chunk % 2) .. + 7
    const int unit = chunk >> 1, h = chunk & 1;
    const u8m val = *reinterpret_cast<const u8m*>(&st[unit * kTrStageStride + 8 * h]);
    *reinterpret_cast<u8m*>(&T[(int64_t)(kUnits * us + unit) * ldT + row0 + 8 * h]) = val;
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

struct TrainRowsArgs {
  const float* P;
  const int32_t* order;
  const int8_t* y;
  int64_t row0;      // first entry of `order` (or row of P) of this batch
  int rows;          // rows in the batch
  int64_t n_rows;    // rows of P
  int d_in;
  const float* mu;
  const float* sd;
  const uint16_t* tw1;   // layer-1 operands [16 v][64 lane][8]
  const float* b1;
  const uint16_t* tw2f;  // layer-2 operands [16 v][8 c][64 lane][8] (W2^T, output units permuted)
  const float* b2;
  const float* w3;
  const float* b3;
  const uint16_t* tw2d;  // dH1 operands [16 v][8 c][64 lane][8] (W2, output units permuted)
  int64_t ldT;           // row stride of the unit-major arrays
  uint16_t* XT;          // [kTrIn][ldT]
  uint16_t* H1T;         // [kTrH][ldT]
  uint16_t* dZ2T;        // [kTrH][ldT]
  uint16_t* dZ1T;        // [kTrH][ldT]
  float* wg_sums;        // [workgroups][kTrVec]
  float* z_out;          // optional logits [rows]
  int* bad;
};

// Copies one 128 KB operand set (kTrH x kTrH bf16) into LDS with a 256-thread
// workgroup, each thread's loads issued 16 at a time.
__device__ __forceinline__ void stage_operands(const uint16_t* __restrict__ g, uint16_t* lds, int tid) {
  const u8m* src = reinterpret_cast<const u8m*>(g);
  u8m* dst = reinterpret_cast<u8m*>(lds);
  constexpr int kPer = kTrH * kTrH / 8 / kTrThreads;  // 16 vectors of 16 bytes per thread
  static_assert(kPer % 16 == 0, "whole groups of 16 loads");
#pragma unroll
  for (int b = 0; b < kPer; b += 16) {
    u8m buf[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) buf[q] = src[(b + q) * kTrThreads + tid];
#pragma unroll
    for (int q = 0; q < 16; ++q) dst[(b + q) * kTrThreads + tid] = buf[q];
  }
}

__global__ void __launch_bounds__(kTrThreads) k_train_rows(TrainRowsArgs a) {
  __shared__ __align__(16) uint16_t w2s[kTrH * kTrH];
  __shared__ __align__(16) float b1s[kTrH], b2s[kTrH], w3s[kTrH];
  __shared__ float sums[kTrBlocks][kTrVec];
  __shared__ float hp[kTrBlocks][kTrSlices][16];  // the head's partial sums of each slice, per row
  __shared__ u4m xch[kTrBlocks][8][64];           // dZ2 in operand form, chunk c of lane l
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, g = lane >> 4, col = lane & 15;
  // row block, unit slice (units 64 us .. + 63); wave-uniform, so that the choices made on them are branches
  const int rb = __builtin_amdgcn_readfirstlane(wave / kTrSlices);
  const int us = __builtin_amdgcn_readfirstlane(wave % kTrSlices);
  stage_operands(a.tw2f, w2s, tid);
  if (tid < kTrH) {
    b1s[tid] = a.b1[tid];
    b2s[tid] = a.b2[tid];
    w3s[tid] = a.w3[tid];
  }
  __syncthreads();
  float* my = sums[rb];
  const int64_t r = (int64_t)blockIdx.x * kTrRows + 16 * rb + col;  // this lane's batch row
  const bool in_batch = r < a.rows;
  int64_t src = -1;
  if (in_batch) {
    const int64_t s = a.order ? (int64_t)a.order[a.row0 + r] : a.row0 + r;
    if (s >= 0 && s < a.n_rows) src = s;
    else if (g == 0 && us == 0) *a.bad = 1;
  }
  const bool live = src >= 0;
  // 1. inputs: features 8 g .. 8 g + 7 of row r (the B operand of layer 1)
  u8m xu;
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const int f = 8 * g + j;
    const float v = (live && f < a.d_in) ? (a.P[src * a.d_in + f] - a.mu[f]) / a.sd[f] : 0.f;
    xu[j] = to_bf16(v);
    if (us == 0) a.XT[(int64_t)f * a.ldT + r] = xu[j];
  }
  const bf8m xb = __builtin_bit_cast(bf8m, xu);
  // 2. layer 1: H1^T = W1^T X^T + b1, ReLU, BF16 (every unit: the operand of layer 2)
  u4m h1[8];
#pragma unroll
  for (int v = 0; v < 16; ++v) {
    const bf8m w = __builtin_bit_cast(bf8m, reinterpret_cast<const u8m*>(a.tw1)[v * 64 + lane]);
    const f4m bias = *reinterpret_cast<const f4m*>(&b1s[32 * (v >> 1) + 8 * g + 4 * (v & 1)]);
    const f4m d = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w, xb, bias, 0, 0, 0);
    h1[v >> 1][2 * (v & 1)] = relu_bf16x2(d[0], d[1]);
    h1[v >> 1][2 * (v & 1) + 1] = relu_bf16x2(d[2], d[3]);
  }
  // 3. layer 2 for this slice's units: Z2^T = W2^T H1^T + b2 (output units permuted like layer 1)
  f4m z2[kTrSliceV];
#pragma unroll
  for (int vv = 0; vv < kTrSliceV; ++vv) {
    const int v = kTrSliceV * us + vv;
    z2[vv] = *reinterpret_cast<const f4m*>(&b2s[32 * (v >> 1) + 8 * g + 4 * (v & 1)]);
  }
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    const bf8m hb = __builtin_bit_cast(bf8m, h1[c]);
#pragma unroll
    for (int vv = 0; vv < kTrSliceV; ++vv) {
      const int v = kTrSliceV * us + vv;
      const bf8m w = __builtin_bit_cast(bf8m, reinterpret_cast<const u8m*>(w2s)[(v * 8 + c) * 64 + lane]);
      z2[vv] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w, hb, z2[vv], 0, 0, 0);
    }
  }
  // 4. head: this slice's partial sum (the four lane groups hold disjoint units of the same row), the
  //    slices' partials added in slice order
  float lp = 0.f;
#pragma unroll
  for (int vv = 0; vv < kTrSliceV; ++vv) {
    const int v = kTrSliceV * us + vv;
    const f4m hw = *reinterpret_cast<const f4m*>(&w3s[32 * (v >> 1) + 8 * g + 4 * (v & 1)]);
#pragma unroll
    for (int i = 0; i < 4; ++i) lp = fmaf(fmaxf(z2[vv][i], 0.f), hw[i], lp);
  }
  lp += __shfl_xor(lp, 16);
  lp += __shfl_xor(lp, 32);
  if (g == 0) hp[rb][us][col] = lp;
  __syncthreads();  // partials visible; every wave is done with the layer-2 operands
  float zs = hp[rb][0][col];
#pragma unroll
  for (int k = 1; k < kTrSlices; ++k) zs += hp[rb][k][col];
  const float z = zs + a.b3[0];
  float dz = 0.f, loss = 0.f;
  if (live) {
    const float t = a.y[src] > 0 ? 1.f : 0.f;
    loss = fmaxf(z, 0.f) + log1pf(expf(-fabsf(z))) - t * z;
    dz = (1.f / (1.f + expf(-z)) - t) / (float)a.rows;
    if (a.z_out && g == 0 && us == 0) a.z_out[r] = z;
  }
  // 5. dZ2 = [Z2 > 0] dz w3 (FP32) for this slice's units, row sums for gb2 and gw3, BF16 copy shared with
  //    the row block's other slices
  u4m d2[kTrSliceC];
#pragma unroll
  for (int vv = 0; vv < kTrSliceV; ++vv) {
    const int v = kTrSliceV * us + vv;
    const int u0 = 32 * (v >> 1) + 8 * g + 4 * (v & 1);
    const f4m hw = *reinterpret_cast<const f4m*>(&w3s[u0]);
    f4m dv;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      dv[i] = z2[vv][i] > 0.f ? dz * hw[i] : 0.f;
      const float sb = rows_sum(dv[i]);
      const float sw = rows_sum(fmaxf(z2[vv][i], 0.f) * dz);
      if (col == 0) {
        my[kTrH + u0 + i] = sb;
        my[2 * kTrH + u0 + i] = sw;
      }
    }
    d2[vv >> 1][2 * (vv & 1)] = pack_bf16x2(dv[0], dv[1]);
    d2[vv >> 1][2 * (vv & 1) + 1] = pack_bf16x2(dv[2], dv[3]);
  }
#pragma unroll
  for (int cc = 0; cc < kTrSliceC; ++cc) xch[rb][kTrSliceC * us + cc][lane] = d2[cc];
  // 6. dH1^T = W2 dZ2^T for this slice's output units (permuted like layer 1), dZ1 = [H1 > 0] dH1; the
  //    LDS operand area now takes the dH1 operands
  stage_operands(a.tw2d, w2s, tid);
  __syncthreads();  // dH1 operands staged, every slice's dZ2 in LDS
  f4m dh[kTrSliceV];
#pragma unroll
  for (int vv = 0; vv < kTrSliceV; ++vv) dh[vv] = (f4m){0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    const bf8m db = __builtin_bit_cast(bf8m, xch[rb][c][lane]);
#pragma unroll
    for (int vv = 0; vv < kTrSliceV; ++vv) {
      const int v = kTrSliceV * us + vv;
      const bf8m w = __builtin_bit_cast(bf8m, reinterpret_cast<const u8m*>(w2s)[(v * 8 + c) * 64 + lane]);
      dh[vv] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w, db, dh[vv], 0, 0, 0);
    }
  }
  // this slice's H1 chunks (the ReLU mask of dZ1, and the rows this wave stores), picked by a uniform branch
  u4m hsl[kTrSliceC];
#pragma unroll
  for (int k = 0; k < kTrSlices; ++k)
    if (us == k)
#pragma unroll
      for (int cc = 0; cc < kTrSliceC; ++cc) hsl[cc] = h1[kTrSliceC * k + cc];
  u4m d1[kTrSliceC];
#pragma unroll
  for (int vv = 0; vv < kTrSliceV; ++vv) {
    const int v = kTrSliceV * us + vv;
    const int u0 = 32 * (v >> 1) + 8 * g + 4 * (v & 1);
    f4m dv;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      dv[i] = bf16_at(hsl[vv >> 1], 4 * (vv & 1) + i) != 0 ? dh[vv][i] : 0.f;
      const float sb = rows_sum(dv[i]);
      if (col == 0) my[u0 + i] = sb;
    }
    d1[vv >> 1][2 * (vv & 1)] = pack_bf16x2(dv[0], dv[1]);
    d1[vv >> 1][2 * (vv & 1) + 1] = pack_bf16x2(dv[2], dv[3]);
  }
  // 7. row sums of dz (gb3) and of the loss (once per row block)
  if (us == 0) {
    const float sdz = rows_sum(g == 0 ? dz : 0.f);
    const float sl = rows_sum(g == 0 ? loss : 0.f);
    if (lane == 0) {
      my[3 * kTrH] = sdz;
      my[3 * kTrH + 1] = sl;
    }
  }
  __syncthreads();  // every wave is done with the dH1 operands: the LDS area now stages the unit-major stores
  {
    const int64_t row0 = (int64_t)blockIdx.x * kTrRows + 16 * rb;
    uint16_t* st = w2s + wave * ((kTrH / kTrSlices) * kTrStageStride);
    store_unit_major(hsl, us, st, a.H1T, a.ldT, row0, lane);
    store_unit_major(d2, us, st, a.dZ2T, a.ldT, row0, lane);
    store_unit_major(d1, us, st, a.dZ1T, a.ldT, row0, lane);
  }
  // workgroup sums in row-block order
  for (int k = tid; k < kTrVec; k += kTrThreads) {
    float s = 0.f;
#pragma unroll
    for (int w = 0; w < kTrBlocks; ++w) s += sums[w][k];
    a.wg_sums[(int64_t)blockIdx.x * kTrVec + k] = s;
  }
}

// gW2 = H1^T dZ2 (tiles 0..31, 32 x 64 outputs) and gW1 = X^T dZ1 (tiles
// 32..35, 32 x 64 outputs), over batch rows [kchunk * split, + kchunk) of the
// unit-major arrays, in groups of 8 row steps of 32 whose operands are all
// loaded before the group's products. One wave per (tile, split); partial
// written to part[split][W1 (kTrIn x kTrH) | W2 (kTrH x kTrH)]. Blocks past
// the tiles sum the per-workgroup vectors of k_train_rows over a contiguous
// range of workgroups per split, in workgroup order, into red[split][kTrVec]
// (the loss sum in FP64 into red_loss[split]).
constexpr int kTrWgradTiles = 36;
constexpr int kTrRedBlocks = (kTrVec + 63) / 64;
__global__ void __launch_bounds__(64) k_train_wgrad(const uint16_t* __restrict__ XT, const uint16_t* __restrict__ H1T,
                                                     const uint16_t* __restrict__ dZ2T,
                                                     const uint16_t* __restrict__ dZ1T, int64_t ldT, int64_t krows,
                                                     int64_t kchunk, float* __restrict__ part,
                                                     const float* __restrict__ wg_sums, int n_wg,
                                                     float* __restrict__ red, double* __restrict__ red_loss) {
  const int lane = threadIdx.x, g = lane >> 4, col = lane & 15;
  const int tile = blockIdx.x, split = blockIdx.y;
  if (tile >= kTrWgradTiles) {
    const int k = (tile - kTrWgradTiles) * 64 + lane;
    if (k >= kTrVec) return;
    const int per = (n_wg + (int)gridDim.y - 1) / (int)gridDim.y;
    const int wa = split * per, wb = wa + per < n_wg ? wa + per : n_wg;
    // workgroups wa .. wb - 1 in order, 16 loads in flight per step; the loss (entry 3 H + 1) also in FP64
    const bool is_loss = k == 3 * kTrH + 1;
    double sd = 0.0;
    float sf = 0.f;
    for (int w0 = wa; w0 < wb; w0 += 16) {
      float buf[16];
#pragma unroll
      for (int q = 0; q < 16; ++q) buf[q] = w0 + q < wb ? wg_sums[(int64_t)(w0 + q) * kTrVec + k] : 0.f;
#pragma unroll
      for (int q = 0; q < 16; ++q) sf += buf[q];
      if (is_loss) {
#pragma unroll
        for (int q = 0; q < 16; ++q) sd += (double)buf[q];
      }
    }
    red[(int64_t)split * kTrVec + k] = sf;
    if (is_loss) red_loss[split] = sd;
    return;
  }
  const bool w2 = tile < 32;
  const uint16_t* A = w2 ? H1T : XT;
  const uint16_t* Bm = w2 ? dZ2T : dZ1T;
  const int m0 = w2 ? 32 * (tile >> 2) : 0;
  const int n0 = w2 ? 64 * (tile & 3) : 64 * (tile - 32);
  f4m acc[2][4];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = (f4m){0.f, 0.f, 0.f, 0.f};
  const int64_t k0 = (int64_t)split * kchunk;
  const int64_t k1 = k0 + kchunk < krows ? k0 + kchunk : krows;
  const u8m* ap[2];
  const u8m* bp[4];
#pragma unroll
  for (int i = 0; i < 2; ++i) ap[i] = reinterpret_cast<const u8m*>(&A[(int64_t)(m0 + 16 * i + col) * ldT + 8 * g]);
#pragma unroll
  for (int j = 0; j < 4; ++j) bp[j] = reinterpret_cast<const u8m*>(&Bm[(int64_t)(n0 + 16 * j + col) * ldT + 8 * g]);
  constexpr int kSteps = 8;
  for (int64_t kg = k0; kg < k1; kg += 32 * kSteps) {
    u8m an[kSteps][2], bn[kSteps][4];
#pragma unroll
    for (int t = 0; t < kSteps; ++t) {
      const int64_t k = kg + 32 * t;
      if (k < k1) {
#pragma unroll
        for (int i = 0; i < 2; ++i) an[t][i] = ap[i][k / 8];
#pragma unroll
        for (int j = 0; j < 4; ++j) bn[t][j] = bp[j][k / 8];
      }
    }
#pragma unroll
    for (int t = 0; t < kSteps; ++t)
      if (kg + 32 * t < k1)
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int j = 0; j < 4; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf8m, an[t][i]),
                                                                __builtin_bit_cast(bf8m, bn[t][j]), acc[i][j], 0, 0, 0);
  }
  float* out = part + (int64_t)split * (kTrIn + kTrH) * kTrH + (w2 ? (int64_t)kTrIn * kTrH : 0);
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int rr = 0; rr < 4; ++rr)
        out[(int64_t)(m0 + 16 * i + 4 * g + rr) * kTrH + n0 + 16 * j + col] = acc[i][j][rr];
}

struct TrainAdamArgs {
  const float* part;     // [splits][(kTrIn + kTrH) * kTrH]
  int splits;
  const float* red;      // [splits][kTrVec] workgroup sums reduced by k_train_wgrad
  const double* red_loss;  // [splits]
  int d_in;
  int64_t n_params;
  float* params;
  float* grads;
  float* m;
  float* v;
  int apply;             // 0: gradients only
  float lr, b1, b2, eps, c1, c2;
  uint16_t* tw1;
  uint16_t* tw2f;
  uint16_t* tw2d;
  uint16_t* w1b;         // staged-path copies [kin_pad][H], [H][H]
  uint16_t* w2b;
  double* loss_acc;
};

// Position of hidden unit u in the permuted MFMA row order (inverse of inf_unit1).
__device__ __forceinline__ void unit_slot(int u, int* v, int* row) {
  *v = 2 * (u >> 5) + ((u & 7) >> 2);
  *row = 4 * ((u & 31) >> 3) + (u & 3);
}

__global__ void __launch_bounds__(256) k_train_adam(TrainAdamArgs a) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e == 0 && a.loss_acc) {
    double l = 0.0;
    for (int sp = 0; sp < a.splits; ++sp) l += a.red_loss[sp];
    *a.loss_acc += l;
  }
  if (e >= a.n_params) return;
  const int64_t nW1 = (int64_t)a.d_in * kTrH;
  const int64_t oW2 = nW1 + kTrH, oB2 = oW2 + (int64_t)kTrH * kTrH, oW3 = oB2 + kTrH, oB3 = oW3 + kTrH;
  const int64_t pstride = (int64_t)(kTrIn + kTrH) * kTrH;
  float gsum = 0.f;
  int kind;  // 0 W1, 1 b1, 2 W2, 3 b2, 4 w3, 5 b3
  int64_t idx;
  if (e < nW1) { kind = 0; idx = e; }
  else if (e < oW2) { kind = 1; idx = e - nW1; }
  else if (e < oB2) { kind = 2; idx = e - oW2; }
  else if (e < oW3) { kind = 3; idx = e - oB2; }
  else if (e < oB3) { kind = 4; idx = e - oW3; }
  else { kind = 5; idx = 0; }
  {
    // split partials in a fixed order, their loads issued 16 at a time
    const bool w = kind == 0 || kind == 2;
    const float* base = w ? a.part + (kind == 0 ? idx : (int64_t)kTrIn * kTrH + idx)
                          : a.red + (kind == 1 ? idx : kind == 3 ? kTrH + idx : kind == 4 ? 2 * kTrH + idx : 3 * kTrH);
    const int64_t stride = w ? pstride : kTrVec;
    for (int s0 = 0; s0 < a.splits; s0 += 16) {
      float buf[16];
#pragma unroll
      for (int q = 0; q < 16; ++q) buf[q] = s0 + q < a.splits ? base[(int64_t)(s0 + q) * stride] : 0.f;
#pragma unroll
      for (int q = 0; q < 16; ++q)
        if (s0 + q < a.splits) gsum += buf[q];
    }
  }
  a.grads[e] = gsum;
  if (!a.apply) return;
  const float mi = a.b1 * a.m[e] + (1.f - a.b1) * gsum;
  const float vi = a.b2 * a.v[e] + (1.f - a.b2) * gsum * gsum;
  a.m[e] = mi;
  a.v[e] = vi;
  const float p = a.params[e] - a.lr * (mi * a.c1) / (sqrtf(vi * a.c2) + a.eps);
  a.params[e] = p;
  const uint16_t pb = to_bf16(p);
  if (kind == 0) {
    const int f = (int)(idx / kTrH), u = (int)(idx % kTrH);
    int v, row;
    unit_slot(u, &v, &row);
    a.tw1[((int64_t)v * 64 + 16 * (f >> 3) + row) * 8 + (f & 7)] = pb;
    a.w1b[idx] = pb;
  } else if (kind == 2) {
    const int u1 = (int)(idx / kTrH), u2 = (int)(idx % kTrH);
    int v, row;
    unit_slot(u2, &v, &row);  // forward operand: rows = u2 (permuted), k = u1
    a.tw2f[(((int64_t)v * 8 + (u1 >> 5)) * 64 + 16 * ((u1 & 31) >> 3) + row) * 8 + (u1 & 7)] = pb;
    unit_slot(u1, &v, &row);  // backward operand: rows = u1 (permuted), k = u2
    a.tw2d[(((int64_t)v * 8 + (u2 >> 5)) * 64 + 16 * ((u2 & 31) >> 3) + row) * 8 + (u2 & 7)] = pb;
    a.w2b[idx] = pb;
  }
}

// Packs all training operands from the FP32 masters (after set_params).
__global__ void __launch_bounds__(256) k_train_pack(const float* __restrict__ w1, const float* __restrict__ w2, int d_in,
                                                     uint16_t* __restrict__ tw1, uint16_t* __restrict__ tw2f,
                                                     uint16_t* __restrict__ tw2d) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  constexpr int64_t n1 = 16 * 64 * 8, n2 = (int64_t)kTrH * kTrH;
  if (e < n1) {
    const int j = (int)(e & 7), lane = (int)((e >> 3) & 63), v = (int)(e >> 9);
    const int k = 8 * (lane >> 4) + j;
    tw1[e] = k < d_in ? to_bf16(w1[(int64_t)k * kTrH + inf_unit1(v, lane & 15)]) : (uint16_t)0;
  } else if (e < n1 + n2) {
    const int64_t f = e - n1;
    const int j = (int)(f & 7), lane = (int)((f >> 3) & 63), c = (int)((f >> 9) & 7), v = (int)(f >> 12);
    const int k = 32 * c + 8 * (lane >> 4) + j;
    const int mrow = inf_unit1(v, lane & 15);
    tw2f[f] = to_bf16(w2[(int64_t)k * kTrH + mrow]);
    tw2d[f] = to_bf16(w2[(int64_t)mrow * kTrH + k]);
  }
}

static inline unsigned nblk(int64_t n) { return (unsigned)((n + 255) / 256); }

}  // namespace fastron

using namespace fastron;

// ---------------------------------------------------------------------------
// Network object
// ---------------------------------------------------------------------------
struct fastron_mlp {
  int d_in = 0, kin_pad = 0, H = 0;
  int64_t n_params = 0;
  int64_t cap_rows = 0;  // capacity of the activation buffers
  float* params = nullptr;  // [w1 d_in*H][b1 H][w2 H*H][b2 H][w3 H][b3 1]
  float* grads = nullptr;
  float* adam_m = nullptr;
  float* adam_v = nullptr;
  float* mu = nullptr;
  float* sd = nullptr;
  uint16_t* w1b = nullptr;  // [kin_pad][H]
  uint16_t* w2b = nullptr;  // [H][H]
  uint16_t* w1p = nullptr;  // fused-inference operand order (H == 256, d_in <= 24 only)
  uint16_t* w2p = nullptr;
  float* isd = nullptr;     // 1 / sd for the fused pass
  // three-kernel training step (H == 256, d_in <= 32)
  bool fast = false;
  int64_t ldT = 0;          // row stride of the unit-major activation arrays
  uint16_t* tw1 = nullptr;
  uint16_t* tw2f = nullptr;
  uint16_t* tw2d = nullptr;
  uint16_t* XT = nullptr;
  uint16_t* H1T = nullptr;
  uint16_t* dZ2T = nullptr;
  uint16_t* dZ1T = nullptr;
  float* wg_sums = nullptr;
  float* wpart = nullptr;
  float* red = nullptr;       // [kTrSplitsMax][kTrVec] reduced workgroup sums per split
  double* red_loss = nullptr;
  double* loss_acc = nullptr;
  float* splitbuf = nullptr;  // split-K partial products of the weight-gradient GEMMs
  int64_t step = 0;
  // activations for a batch of cap_rows
  uint16_t* Xb = nullptr;
  float* Z1 = nullptr;
  uint16_t* H1b = nullptr;
  float* Z2 = nullptr;
  float* partial = nullptr;
  float* z = nullptr;
  float* dz = nullptr;
  float* dZ2 = nullptr;
  uint16_t* dZ2b = nullptr;
  float* dH1 = nullptr;
  float* dZ1 = nullptr;
  uint16_t* dZ1b = nullptr;
  float* colpart = nullptr;
  float* loss_part = nullptr;
  float* hbuf = nullptr;  // relu(Z2)
  int* bad = nullptr;     // set by kernels that met an out-of-range row index
  float* w1() { return params; }
  float* b1() { return params + (int64_t)d_in * H; }
  float* w2() { return b1() + H; }
  float* b2() { return w2() + (int64_t)H * H; }
  float* w3() { return b2() + H; }
  float* b3() { return w3() + H; }
};

namespace {

int64_t param_count(int d_in, int H) { return (int64_t)d_in * H + H + (int64_t)H * H + H + H + 1; }

void free_mlp(fastron_mlp* n) {
  if (!n) return;
  void* ps[] = {n->params, n->grads, n->adam_m, n->adam_v, n->mu, n->sd, n->w1b, n->w2b, n->Xb, n->Z1, n->H1b,
                n->Z2, n->partial, n->z, n->dz, n->dZ2, n->dZ2b, n->dH1, n->dZ1, n->dZ1b, n->colpart, n->loss_part,
                n->hbuf, n->bad, n->w1p, n->w2p, n->isd, n->splitbuf, n->tw1, n->tw2f, n->tw2d, n->XT,
                n->H1T, n->dZ2T, n->dZ1T, n->wg_sums, n->wpart, n->loss_acc, n->red, n->red_loss};
  for (void* p : ps) (void)hipFree(p);
  delete n;
}

constexpr int64_t kSplitFloats = 4 << 20;  // split-K workspace (16 MB)

// C = act(A B + bias). Output grids too small to fill the device (the weight
// gradients: a few 64 x 64 tiles, K = batch rows) split K across blockIdx.z
// into `split` (kSplitFloats floats) and reduce in a second kernel.
fastron_status gemm(hipStream_t s, const uint16_t* A, int64_t sam, int64_t sak, const uint16_t* B, int64_t sbk,
                    int64_t sbn, int M, int N, int K, float* C, int64_t ldc, uint16_t* Cb, int64_t ldcb,
                    const float* bias, int relu, const float* head = nullptr, float* partial = nullptr,
                    float* split = nullptr) {
  const int64_t tiles = (int64_t)((M + kGT - 1) / kGT) * ((N + kGT - 1) / kGT);
  int64_t splits = 1;
  if (split && !head && tiles < 128 && K >= 4 * 128) {
    splits = (512 + tiles - 1) / tiles;
    const int64_t by_k = K / 128;  // at least 128 rows of K per split
    const int64_t by_mem = kSplitFloats / ((int64_t)M * N);
    if (splits > by_k) splits = by_k;
    if (splits > by_mem) splits = by_mem;
    if (splits < 1) splits = 1;
  }
  int64_t kchunk = (K + splits - 1) / splits;
  kchunk = (kchunk + kGK - 1) / kGK * kGK;
  if (kchunk < kGK) kchunk = kGK;
  splits = (K + kchunk - 1) / kchunk;
  if (splits < 1) splits = 1;
  GemmArgs g{A, sam, sak, B, sbk, sbn, C, ldc, Cb, ldcb, bias, head, partial, relu, M, N, K, (int)kchunk,
             splits > 1 ? split : nullptr};
  dim3 grid((unsigned)((M + kGT - 1) / kGT), (unsigned)((N + kGT - 1) / kGT), (unsigned)splits);
  hipLaunchKernelGGL(k_gemm_bf16, grid, dim3(256), 0, s, g);
  FASTRON_HIP(hipGetLastError());
  if (splits > 1) {
    hipLaunchKernelGGL(k_splitk_reduce, dim3((unsigned)(((int64_t)M * N + 255) / 256)), dim3(256), 0, s, split,
                       (int)splits, M, N, bias, relu, C, ldc, Cb, ldcb);
    FASTRON_HIP(hipGetLastError());
  }
  return FASTRON_OK;
}

fastron_status colsum(hipStream_t s, fastron_mlp* n, const float* X, int64_t rows, int cols, int64_t ld,
                      const float* scale, float* out) {
  dim3 g1((unsigned)((cols + 255) / 256), kColChunks);
  hipLaunchKernelGGL(k_colsum_pass1, g1, dim3(256), 0, s, X, rows, cols, ld, scale, n->colpart);
  FASTRON_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_colsum_pass2, dim3((unsigned)((cols + 255) / 256)), dim3(256), 0, s, n->colpart, cols, out);
  FASTRON_HIP(hipGetLastError());
  return FASTRON_OK;
}

#define TRY(x)                                   \
  do {                                           \
    fastron_status st_ = (x);                    \
    if (st_ != FASTRON_OK) return st_;           \
  } while (0)

// Forward over `rows` rows already staged in Xb; fills Z1, H1b, Z2 and the logits z.
fastron_status forward_staged(fastron_mlp* n, int64_t rows, bool keep, hipStream_t s) {
  const int H = n->H;
  // layer 1: Z1 = X W1 + b1, H1 = relu(Z1)
  TRY(gemm(s, n->Xb, n->kin_pad, 1, n->w1b, H, 1, (int)rows, H, n->kin_pad, keep ? n->Z1 : nullptr, H, n->H1b, H,
           n->b1(), 1));
  // layer 2 (+ fused head): Z2 = H1 W2 + b2; partial = relu(Z2) . w3 per 64-column tile
  TRY(gemm(s, n->H1b, H, 1, n->w2b, H, 1, (int)rows, H, H, keep ? n->Z2 : nullptr, H, nullptr, 0, n->b2(), 1,
           n->w3(), n->partial));
  const int ntile = (H + kGT - 1) / kGT;
  hipLaunchKernelGGL(k_head_forward, dim3(nblk(rows)), dim3(256), 0, s, n->partial, ntile, rows, n->b3(), n->z);
  FASTRON_HIP(hipGetLastError());
  return FASTRON_OK;
}

// Gradients of the mean BCE over the staged rows into n->grads (Z1, Z2 must be kept).
fastron_status backward(fastron_mlp* n, int64_t rows, const int8_t* y, const int32_t* order, int64_t row0,
                        int64_t n_rows, hipStream_t s) {
  const int H = n->H;
  float* g = n->grads;
  float* gw1 = g;
  float* gb1 = g + (int64_t)n->d_in * H;
  float* gw2 = gb1 + H;
  float* gb2 = gw2 + (int64_t)H * H;
  float* gw3 = gb2 + H;
  float* gb3 = gw3 + H;
  hipLaunchKernelGGL(k_bce, dim3(nblk(rows)), dim3(256), 0, s, n->z, y, order, row0, rows, n_rows, n->dz,
                     n->loss_part);
  FASTRON_HIP(hipGetLastError());
  // last layer: gw3 = relu(Z2)^T dz, gb3 = sum dz
  hipLaunchKernelGGL(k_relu_copy, dim3(nblk(rows * H)), dim3(256), 0, s, n->Z2, rows * H, n->hbuf);
  FASTRON_HIP(hipGetLastError());
  TRY(colsum(s, n, n->hbuf, rows, H, H, n->dz, gw3));
  TRY(colsum(s, n, n->dz, rows, 1, 1, nullptr, gb3));
  // layer 2: dZ2 = dz w3 [Z2 > 0]; gW2 = H1^T dZ2; gb2 = sum dZ2
  hipLaunchKernelGGL(k_head_back, dim3(nblk(rows * H)), dim3(256), 0, s, n->dz, n->w3(), n->Z2, rows, H, n->dZ2,
                     n->dZ2b);
  FASTRON_HIP(hipGetLastError());
  TRY(gemm(s, n->H1b, 1, H, n->dZ2b, H, 1, H, H, (int)rows, gw2, H, nullptr, 0, nullptr, 0, nullptr, nullptr,
           n->splitbuf));
  TRY(colsum(s, n, n->dZ2, rows, H, H, nullptr, gb2));
  // layer 1: dH1 = dZ2 W2^T; dZ1 = dH1 [Z1 > 0]; gW1 = X^T dZ1; gb1 = sum dZ1
  TRY(gemm(s, n->dZ2b, H, 1, n->w2b, 1, H, (int)rows, H, H, n->dH1, H, nullptr, 0, nullptr, 0));
  hipLaunchKernelGGL(k_relu_back, dim3(nblk(rows * H)), dim3(256), 0, s, n->dH1, n->Z1, rows * H, n->dZ1, n->dZ1b);
  FASTRON_HIP(hipGetLastError());
  TRY(gemm(s, n->Xb, 1, n->kin_pad, n->dZ1b, H, 1, n->d_in, H, (int)rows, gw1, H, nullptr, 0, nullptr, 0, nullptr,
           nullptr, n->splitbuf));
  TRY(colsum(s, n, n->dZ1, rows, H, H, nullptr, gb1));
  return FASTRON_OK;
}

fastron_status refresh_bf16(fastron_mlp* n, hipStream_t s) {
  const int64_t tot = (int64_t)n->kin_pad * n->H + (int64_t)n->H * n->H;
  hipLaunchKernelGGL(k_weights_bf16, dim3(nblk(tot)), dim3(256), 0, s, n->w1(), n->w2(), n->d_in, n->kin_pad, n->H,
                     n->w1b, n->w2b);
  FASTRON_HIP(hipGetLastError());
  if (n->fast) {
    hipLaunchKernelGGL(k_train_pack, dim3(nblk(16 * 64 * 8 + (int64_t)kTrH * kTrH)), dim3(256), 0, s, n->w1(), n->w2(),
                       n->d_in, n->tw1, n->tw2f, n->tw2d);
    FASTRON_HIP(hipGetLastError());
  }
  return FASTRON_OK;
}

// One batch of the three-kernel step on rows row0 .. row0 + rows - 1 of
// `order` (or of P): gradients into n->grads and, with apply, an Adam step
// that also refreshes every BF16 operand copy. The batch's loss sum is added
// to n->loss_acc.
fastron_status fast_step(fastron_mlp* n, const float* P, const int8_t* y, const int32_t* order, int64_t row0,
                         int64_t rows, int64_t n_rows, bool apply, float lr, float* z_out, hipStream_t s) {
  const int nwg = (int)((rows + kTrRows - 1) / kTrRows);
  TrainRowsArgs a;
  a.P = P;
  a.order = order;
  a.y = y;
  a.row0 = row0;
  a.rows = (int)rows;
  a.n_rows = n_rows;
  a.d_in = n->d_in;
  a.mu = n->mu;
  a.sd = n->sd;
  a.tw1 = n->tw1;
  a.b1 = n->b1();
  a.tw2f = n->tw2f;
  a.b2 = n->b2();
  a.w3 = n->w3();
  a.b3 = n->b3();
  a.tw2d = n->tw2d;
  a.ldT = n->ldT;
  a.XT = n->XT;
  a.H1T = n->H1T;
  a.dZ2T = n->dZ2T;
  a.dZ1T = n->dZ1T;
  a.wg_sums = n->wg_sums;
  a.z_out = z_out;
  a.bad = n->bad;
  hipLaunchKernelGGL(k_train_rows, dim3((unsigned)nwg), dim3(kTrThreads), 0, s, a);
  FASTRON_HIP(hipGetLastError());
  const int64_t krows = (int64_t)nwg * kTrRows;
  int64_t splits = krows / 256;  // about 8 row steps of 32 per wave
  if (splits < 1) splits = 1;
  if (splits > kTrSplitsMax) splits = kTrSplitsMax;
  int64_t kchunk = (krows / 32 + splits - 1) / splits * 32;
  splits = (krows + kchunk - 1) / kchunk;
  hipLaunchKernelGGL(k_train_wgrad, dim3(kTrWgradTiles + kTrRedBlocks, (unsigned)splits), dim3(64), 0, s, n->XT,
                     n->H1T, n->dZ2T, n->dZ1T, n->ldT, krows, kchunk, n->wpart, n->wg_sums, nwg, n->red,
                     n->red_loss);
  FASTRON_HIP(hipGetLastError());
  TrainAdamArgs m;
  m.part = n->wpart;
  m.splits = (int)splits;
  m.red = n->red;
  m.red_loss = n->red_loss;
  m.d_in = n->d_in;
  m.n_params = n->n_params;
  m.params = n->params;
  m.grads = n->grads;
  m.m = n->adam_m;
  m.v = n->adam_v;
  m.apply = apply ? 1 : 0;
  m.lr = lr;
  m.b1 = 0.9f;
  m.b2 = 0.999f;
  m.eps = 1e-8f;
  if (apply) n->step += 1;
  m.c1 = apply ? (float)(1.0 / (1.0 - std::pow((double)m.b1, (double)n->step))) : 0.f;
  m.c2 = apply ? (float)(1.0 / (1.0 - std::pow((double)m.b2, (double)n->step))) : 0.f;
  m.tw1 = n->tw1;
  m.tw2f = n->tw2f;
  m.tw2d = n->tw2d;
  m.w1b = n->w1b;
  m.w2b = n->w2b;
  m.loss_acc = n->loss_acc;
  hipLaunchKernelGGL(k_train_adam, dim3(nblk(n->n_params)), dim3(256), 0, s, m);
  FASTRON_HIP(hipGetLastError());
  return FASTRON_OK;
}

__global__ void k_zero_f64(double* p) {
  if (threadIdx.x == 0) *p = 0.0;
}

fastron_status stage_points(fastron_mlp* n, const float* P, const int32_t* order, int64_t row0, int64_t rows,
                            int64_t n_rows, hipStream_t s) {
  hipLaunchKernelGGL(k_mlp_input_points, dim3(nblk(rows * n->kin_pad)), dim3(256), 0, s, P, order, row0, rows,
                     n_rows, n->d_in, n->kin_pad, n->mu, n->sd, n->Xb, nullptr, n->bad);
  FASTRON_HIP(hipGetLastError());
  return FASTRON_OK;
}

// Fused screening pass (hidden width 256, input width <= 24): packs the
// operands, then one persistent launch sized to the resident capacity.
fastron_status screen_fused(fastron_mlp* n, const ChainArgs& c, const float* q, int64_t N, float tau, float* logits,
                            int8_t* label, uint8_t* fell_back, int32_t* fb_idx, unsigned long long* count,
                            hipStream_t s) {
  const int64_t tot = 16 * 64 * 8 + (int64_t)kInfH * kInfH;
  hipLaunchKernelGGL(k_pack_infer, dim3(nblk(tot)), dim3(256), 0, s, n->w1(), n->w2(), n->sd, n->d_in, n->w1p,
                     n->w2p, n->isd);
  FASTRON_HIP(hipGetLastError());
  InferArgs a;
  a.c = c;
  a.q = q;
  a.N = N;
  a.ntiles = (N + kInfTile - 1) / kInfTile;
  a.mu = n->mu;
  a.isd = n->isd;
  a.w1p = n->w1p;
  a.b1 = n->b1();
  a.w2p = n->w2p;
  a.b2 = n->b2();
  a.w3 = n->w3();
  a.b3 = n->b3();
  a.tau = tau;
  a.logit = logits;
  a.label = label;
  a.fell_back = fell_back;
  a.fb_idx = fb_idx;
  a.fb_count = count;
  // FP32 chain with hardware sin / cos for the network's features at any n:
  // they are rounded to BF16 (2^-9 relative) right after, far coarser than
  // the chain's error.
  const void* kfn = reinterpret_cast<const void*>(k_mlp_screen_fused);
  int dev = 0, ncu = 0, per_cu = 0;
  FASTRON_HIP(hipGetDevice(&dev));
  FASTRON_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
  FASTRON_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kfn, kInfTile, 0));
  if (per_cu < 1) return fail(FASTRON_EUNSUPPORTED, "fused screening kernel cannot be resident");
  int64_t grid = (int64_t)ncu * per_cu;
  if (grid > a.ntiles) grid = a.ntiles;
  void* args[] = {&a};
  FASTRON_HIP(hipLaunchKernel(kfn, dim3((unsigned)grid), dim3(kInfTile), args, 0, s));
  return FASTRON_OK;
}

}  // namespace

extern "C" {

fastron_status fastron_mlp_create(int32_t d_in, int32_t hidden, int64_t max_rows, fastron_mlp** out) {
  clear_error();
  FASTRON_CHECK(out != nullptr, "out is NULL");
  *out = nullptr;
  FASTRON_CHECK(d_in >= 1 && d_in <= 3 * FASTRON_MAX_POINTS, "d_in = %d outside [1, %d]", d_in,
                3 * FASTRON_MAX_POINTS);
  FASTRON_CHECK(hidden >= 16 && hidden <= 1024 && hidden % 16 == 0, "hidden = %d must be a multiple of 16 in [16, 1024]",
                hidden);
  FASTRON_CHECK(max_rows >= 1 && max_rows <= (1ll << 24), "max_rows = %lld outside [1, 2^24]", (long long)max_rows);
  fastron_mlp* n = new fastron_mlp();
  n->d_in = d_in;
  n->kin_pad = (d_in + 31) / 32 * 32;
  n->H = hidden;
  n->n_params = param_count(d_in, hidden);
  n->cap_rows = max_rows;
  const int64_t R = max_rows, H = hidden;
  hipError_t e = hipSuccess;
  auto alloc = [&](auto** p, int64_t count, size_t elem) {
    if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(p), (size_t)(count > 0 ? count : 1) * elem);
  };
  alloc(&n->params, n->n_params, 4);
  alloc(&n->grads, n->n_params, 4);
  alloc(&n->adam_m, n->n_params, 4);
  alloc(&n->adam_v, n->n_params, 4);
  alloc(&n->mu, d_in, 4);
  alloc(&n->sd, d_in, 4);
  alloc(&n->w1b, n->kin_pad * H, 2);
  alloc(&n->w2b, H * H, 2);
  alloc(&n->Xb, R * n->kin_pad, 2);
  alloc(&n->Z1, R * H, 4);
  alloc(&n->H1b, R * H, 2);
  alloc(&n->Z2, R * H, 4);
  alloc(&n->partial, R * ((H + kGT - 1) / kGT), 4);
  alloc(&n->z, R, 4);
  alloc(&n->dz, R, 4);
  alloc(&n->dZ2, R * H, 4);
  alloc(&n->dZ2b, R * H, 2);
  alloc(&n->dH1, R * H, 4);
  alloc(&n->dZ1, R * H, 4);
  alloc(&n->dZ1b, R * H, 2);
  alloc(&n->colpart, (int64_t)kColChunks * H, 4);
  alloc(&n->loss_part, (R + 255) / 256, 4);
  alloc(&n->hbuf, R * H, 4);
  alloc(&n->bad, 1, 4);
  alloc(&n->splitbuf, kSplitFloats, 4);
  if (hidden == kInfH && d_in <= kInfXRow) {
    alloc(&n->w1p, 16 * 64 * 8, 2);
    alloc(&n->w2p, (int64_t)kInfH * kInfH, 2);
    alloc(&n->isd, d_in, 4);
  }
  if (hidden == kTrH && d_in <= kTrIn) {
    n->fast = true;
    n->ldT = (R + kTrRows - 1) / kTrRows * kTrRows;
    alloc(&n->tw1, 16 * 64 * 8, 2);
    alloc(&n->tw2f, (int64_t)kTrH * kTrH, 2);
    alloc(&n->tw2d, (int64_t)kTrH * kTrH, 2);
    alloc(&n->XT, (int64_t)kTrIn * n->ldT, 2);
    alloc(&n->H1T, (int64_t)kTrH * n->ldT, 2);
    alloc(&n->dZ2T, (int64_t)kTrH * n->ldT, 2);
    alloc(&n->dZ1T, (int64_t)kTrH * n->ldT, 2);
    alloc(&n->wg_sums, (n->ldT / kTrRows) * kTrVec, 4);
    alloc(&n->wpart, (int64_t)kTrSplitsMax * (kTrIn + kTrH) * kTrH, 4);
    alloc(&n->loss_acc, 1, 8);
    alloc(&n->red, (int64_t)kTrSplitsMax * kTrVec, 4);
    alloc(&n->red_loss, kTrSplitsMax, 8);
  }
  if (e == hipSuccess) e = hipMemset(n->adam_m, 0, n->n_params * 4);
  if (e == hipSuccess) e = hipMemset(n->adam_v, 0, n->n_params * 4);
  if (e == hipSuccess) e = hipMemset(n->bad, 0, sizeof(int));
  if (e != hipSuccess) {
    free_mlp(n);
    return fail(e == hipErrorOutOfMemory ? FASTRON_ENOMEM : FASTRON_EHIP, "MLP allocation failed: %s",
                hipGetErrorString(e));
  }
  *out = n;
  return FASTRON_OK;
}

void fastron_mlp_destroy(fastron_mlp* n) { free_mlp(n); }

int64_t fastron_mlp_param_count(const fastron_mlp* n) { return n ? n->n_params : -1; }

fastron_status fastron_mlp_set_params(fastron_mlp* n, const float* params, const float* mu, const float* sd,
                                      void* stream) {
  clear_error();
  FASTRON_CHECK(n && params, "network and params must be non-NULL");
  hipStream_t s = as_stream(stream);
  FASTRON_HIP(hipMemcpyAsync(n->params, params, n->n_params * 4, hipMemcpyDeviceToDevice, s));
  if (mu) FASTRON_HIP(hipMemcpyAsync(n->mu, mu, n->d_in * 4, hipMemcpyDeviceToDevice, s));
  if (sd) FASTRON_HIP(hipMemcpyAsync(n->sd, sd, n->d_in * 4, hipMemcpyDeviceToDevice, s));
  FASTRON_HIP(hipMemsetAsync(n->adam_m, 0, n->n_params * 4, s));
  FASTRON_HIP(hipMemsetAsync(n->adam_v, 0, n->n_params * 4, s));
  n->step = 0;
  return refresh_bf16(n, s);
}

fastron_status fastron_mlp_get_params(const fastron_mlp* n, float* params, float* grads, float* mu, float* sd,
                                      void* stream) {
  clear_error();
  FASTRON_CHECK(n != nullptr, "network is NULL");
  hipStream_t s = as_stream(stream);
  if (params) FASTRON_HIP(hipMemcpyAsync(params, n->params, n->n_params * 4, hipMemcpyDeviceToDevice, s));
  if (grads) FASTRON_HIP(hipMemcpyAsync(grads, n->grads, n->n_params * 4, hipMemcpyDeviceToDevice, s));
  if (mu) FASTRON_HIP(hipMemcpyAsync(mu, n->mu, n->d_in * 4, hipMemcpyDeviceToDevice, s));
  if (sd) FASTRON_HIP(hipMemcpyAsync(sd, n->sd, n->d_in * 4, hipMemcpyDeviceToDevice, s));
  return FASTRON_OK;
}

fastron_status fastron_mlp_get_adam_state(const fastron_mlp* n, float* m, float* v, int64_t* step, void* stream) {
  clear_error();
  FASTRON_CHECK(n != nullptr, "network is NULL");
  hipStream_t s = as_stream(stream);
  if (m) FASTRON_HIP(hipMemcpyAsync(m, n->adam_m, n->n_params * 4, hipMemcpyDeviceToDevice, s));
  if (v) FASTRON_HIP(hipMemcpyAsync(v, n->adam_v, n->n_params * 4, hipMemcpyDeviceToDevice, s));
  if (step) *step = n->step;
  return FASTRON_OK;
}

fastron_status fastron_mlp_fit_standardisation(fastron_mlp* n, const float* P, int64_t N, void* stream) {
  clear_error();
  FASTRON_CHECK(n && P, "network and P must be non-NULL");
  FASTRON_CHECK(N >= 1, "N < 1");
  hipLaunchKernelGGL(k_feat_stats, dim3((unsigned)n->d_in), dim3(256), 0, as_stream(stream), P, N, n->d_in, n->mu,
                     n->sd);
  FASTRON_HIP(hipGetLastError());
  return FASTRON_OK;
}

fastron_status fastron_mlp_forward(fastron_mlp* n, const float* P, int64_t N, float* logits, void* stream) {
  clear_error();
  FASTRON_CHECK(n && (N == 0 || (P && logits)), "network, P and logits must be non-NULL");
  FASTRON_CHECK(N >= 0, "N < 0");
  hipStream_t s = as_stream(stream);
  for (int64_t r0 = 0; r0 < N; r0 += n->cap_rows) {
    const int64_t rows = N - r0 < n->cap_rows ? N - r0 : n->cap_rows;
    TRY(stage_points(n, P, nullptr, r0, rows, N, s));
    TRY(forward_staged(n, rows, false, s));
    FASTRON_HIP(hipMemcpyAsync(logits + r0, n->z, rows * 4, hipMemcpyDeviceToDevice, s));
  }
  return FASTRON_OK;
}

fastron_status fastron_mlp_gradients(fastron_mlp* n, const float* P, const int8_t* y, int64_t N, float* loss,
                                     void* stream) {
  clear_error();
  FASTRON_CHECK(n && P && y, "network, P and y must be non-NULL");
  FASTRON_CHECK(N >= 1 && N <= n->cap_rows, "N = %lld outside [1, max_rows]", (long long)N);
  hipStream_t s = as_stream(stream);
  if (n->fast) {
    hipLaunchKernelGGL(k_zero_f64, dim3(1), dim3(64), 0, s, n->loss_acc);
    FASTRON_HIP(hipGetLastError());
    TRY(fast_step(n, P, y, nullptr, 0, N, N, false, 0.f, nullptr, s));
    if (loss) {
      double acc = 0.0;
      FASTRON_HIP(hipMemcpyAsync(&acc, n->loss_acc, sizeof(double), hipMemcpyDeviceToHost, s));
      FASTRON_HIP(hipStreamSynchronize(s));
      *loss = (float)(acc / (double)N);
    }
    return FASTRON_OK;
  }
  TRY(stage_points(n, P, nullptr, 0, N, N, s));
  TRY(forward_staged(n, N, true, s));
  TRY(backward(n, N, y, nullptr, 0, N, s));
  if (loss) {
    const int nb = (int)((N + 255) / 256);
    std::vector<float> lp(nb);
    FASTRON_HIP(hipMemcpyAsync(lp.data(), n->loss_part, nb * 4, hipMemcpyDeviceToHost, s));
    FASTRON_HIP(hipStreamSynchronize(s));
    double acc = 0.0;
    for (float v : lp) acc += v;
    *loss = (float)(acc / (double)N);
  }
  return FASTRON_OK;
}

fastron_status fastron_mlp_train_epoch(fastron_mlp* n, const float* P, const int8_t* y, const int32_t* order,
                                       int64_t N, int64_t batch, float lr, float* mean_loss, void* stream) {
  clear_error();
  FASTRON_CHECK(n && P && y, "network, P and y must be non-NULL");
  FASTRON_CHECK(N >= 1 && batch >= 1 && batch <= n->cap_rows, "need N >= 1 and 1 <= batch <= max_rows");
  FASTRON_CHECK(std::isfinite(lr) && lr > 0.f, "lr must be > 0");
  hipStream_t s = as_stream(stream);
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  FASTRON_HIP(hipMemsetAsync(n->bad, 0, sizeof(int), s));
  if (n->fast) {
    // three kernels per batch, the loss summed on the device; one synchronisation per epoch
    hipLaunchKernelGGL(k_zero_f64, dim3(1), dim3(64), 0, s, n->loss_acc);
    FASTRON_HIP(hipGetLastError());
    for (int64_t r0 = 0; r0 < N; r0 += batch) {
      const int64_t rows = N - r0 < batch ? N - r0 : batch;
      TRY(fast_step(n, P, y, order, r0, rows, N, true, lr, nullptr, s));
    }
    struct {
      double loss;
      int bad;
    } h{0.0, 0};
    FASTRON_HIP(hipMemcpyAsync(&h.loss, n->loss_acc, sizeof(double), hipMemcpyDeviceToHost, s));
    FASTRON_HIP(hipMemcpyAsync(&h.bad, n->bad, sizeof(int), hipMemcpyDeviceToHost, s));
    FASTRON_HIP(hipStreamSynchronize(s));
    if (h.bad) return fail(FASTRON_EINVAL, "order holds a row index outside [0, N)");
    if (mean_loss) *mean_loss = (float)(h.loss / (double)N);
    return FASTRON_OK;
  }
  std::vector<float> lp;
  double loss_acc = 0.0;
  for (int64_t r0 = 0; r0 < N; r0 += batch) {
    const int64_t rows = N - r0 < batch ? N - r0 : batch;
    TRY(stage_points(n, P, order, r0, rows, N, s));
    TRY(forward_staged(n, rows, true, s));
    TRY(backward(n, rows, y, order, r0, N, s));
    n->step += 1;
    const float c1 = (float)(1.0 / (1.0 - std::pow((double)b1, (double)n->step)));
    const float c2 = (float)(1.0 / (1.0 - std::pow((double)b2, (double)n->step)));
    hipLaunchKernelGGL(k_adam, dim3(nblk(n->n_params)), dim3(256), 0, s, n->params, n->grads, n->adam_m, n->adam_v,
                       n->n_params, lr, b1, b2, eps, c1, c2);
    FASTRON_HIP(hipGetLastError());
    TRY(refresh_bf16(n, s));
    if (mean_loss) {
      const int nb = (int)((rows + 255) / 256);
      lp.resize(nb);
      FASTRON_HIP(hipMemcpyAsync(lp.data(), n->loss_part, nb * 4, hipMemcpyDeviceToHost, s));
      FASTRON_HIP(hipStreamSynchronize(s));
      for (float v : lp) loss_acc += v;
    }
  }
  int h_bad = 0;
  FASTRON_HIP(hipMemcpyAsync(&h_bad, n->bad, sizeof(int), hipMemcpyDeviceToHost, s));
  FASTRON_HIP(hipStreamSynchronize(s));
  if (h_bad) return fail(FASTRON_EINVAL, "order holds a row index outside [0, N)");
  if (mean_loss) *mean_loss = (float)(loss_acc / (double)N);
  return FASTRON_OK;
}

fastron_status fastron_mlp_screen(fastron_mlp* n, const fastron_chain* chain, const fastron_cpoints* cp,
                                  const fastron_model* model, const float* q, int64_t N, float tau, float* logits,
                                  int8_t* label, uint8_t* fell_back, int64_t* n_fallback, void* workspace,
                                  int64_t workspace_bytes, void* stream) {
  clear_error();
  ChainArgs c;
  fastron_status st = pack_chain(chain, cp, &c, true);
  if (st != FASTRON_OK) return st;
  FASTRON_CHECK(n != nullptr, "network is NULL");
  FASTRON_CHECK(3 * c.M == n->d_in, "network input width %d != 3 M = %d", n->d_in, 3 * c.M);
  FASTRON_CHECK(N >= 0, "N < 0");
  FASTRON_CHECK(N == 0 || (q && label), "q and label must be non-NULL");
  FASTRON_CHECK(std::isfinite(tau) && tau >= 0.f, "tau must be >= 0");
  FASTRON_CHECK(model != nullptr && model->M == c.M, "model missing or prepared for another M");
  FASTRON_CHECK(N < INT32_MAX, "N too large");
  const int64_t need = 256 + N * 4 + N * (int64_t)c.n * 4 + N * 5;
  FASTRON_CHECK(workspace && workspace_bytes >= need, "workspace needs %lld bytes", (long long)need);
  hipStream_t s = as_stream(stream);
  char* ws = static_cast<char*>(workspace);
  unsigned long long* count = reinterpret_cast<unsigned long long*>(ws);
  int32_t* fb_idx = reinterpret_cast<int32_t*>(ws + 256);
  float* q_sub = reinterpret_cast<float*>(ws + 256 + N * 4);
  float* f_sub = reinterpret_cast<float*>(ws + 256 + N * 4 + N * (int64_t)c.n * 4);
  int8_t* l_sub = reinterpret_cast<int8_t*>(ws + 256 + N * 8 + N * (int64_t)c.n * 4);
  hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, s, count);
  FASTRON_HIP(hipGetLastError());
  if (n->w1p && N > 0) {
    TRY(screen_fused(n, c, q, N, tau, logits, label, fell_back, fb_idx, count, s));
  } else
  for (int64_t r0 = 0; r0 < N; r0 += n->cap_rows) {
    const int64_t rows = N - r0 < n->cap_rows ? N - r0 : n->cap_rows;
    if (c.n >= kFp64Joints)
      hipLaunchKernelGGL(k_mlp_input_fk<double>, dim3(nblk(rows)), dim3(256), 0, s, c, q, r0, rows, n->kin_pad, n->mu,
                         n->sd, n->Xb);
    else
      hipLaunchKernelGGL(k_mlp_input_fk<float>, dim3(nblk(rows)), dim3(256), 0, s, c, q, r0, rows, n->kin_pad, n->mu,
                         n->sd, n->Xb);
    FASTRON_HIP(hipGetLastError());
    TRY(forward_staged(n, rows, false, s));
    hipLaunchKernelGGL(k_screen, dim3(nblk(rows)), dim3(256), 0, s, n->z, r0, rows, tau, logits, label, fell_back,
                       fb_idx, count);
    FASTRON_HIP(hipGetLastError());
  }
  unsigned long long h_count = 0;
  FASTRON_HIP(hipMemcpyAsync(&h_count, count, 8, hipMemcpyDeviceToHost, s));
  FASTRON_HIP(hipStreamSynchronize(s));
  if (n_fallback) *n_fallback = (int64_t)h_count;
  if (h_count == 0) return FASTRON_OK;
  hipLaunchKernelGGL(k_gather_rows, dim3(nblk((int64_t)h_count * c.n)), dim3(256), 0, s, q, c.n, fb_idx, count, q_sub);
  FASTRON_HIP(hipGetLastError());
  st = fastron_fk_score_prepared(chain, cp, model, q_sub, (int64_t)h_count, f_sub, l_sub, FASTRON_SCORE_FP32, stream);
  if (st != FASTRON_OK) return st;
  hipLaunchKernelGGL(k_scatter_labels, dim3(nblk((int64_t)h_count)), dim3(256), 0, s, l_sub, f_sub, fb_idx, count,
                     label, nullptr);
  FASTRON_HIP(hipGetLastError());
  return FASTRON_OK;
}

int64_t fastron_mlp_screen_workspace_bytes(int64_t N, int32_t n_joints) {
  if (N < 0 || n_joints < 1) return -1;
  return 256 + N * 4 + N * (int64_t)n_joints * 4 + N * 5;
}

}  // extern "C"
