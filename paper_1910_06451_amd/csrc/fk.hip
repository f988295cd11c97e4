// Forward kinematics (Section II-A, Eq. 1-2), the prepared support set and the
// library's shared host utilities (errors, argument packing).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>

#include "fastron_internal.h"
#include "model_layout.h"

namespace fastron {

// ---------------------------------------------------------------------------
// Errors
// ---------------------------------------------------------------------------
static thread_local char g_err[512];

void clear_error() { g_err[0] = '\0'; }

fastron_status fail(fastron_status st, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
  return st;
}

// ---------------------------------------------------------------------------
// Chain packing and validation (host only, no HIP calls)
// ---------------------------------------------------------------------------
fastron_status pack_chain(const fastron_chain* chain, const fastron_cpoints* cp, ChainArgs* out, bool need_points) {
  FASTRON_CHECK(chain != nullptr, "chain is NULL");
  FASTRON_CHECK(chain->n >= 1 && chain->n <= FASTRON_MAX_JOINTS, "chain->n = %d outside [1, %d]", chain->n,
                FASTRON_MAX_JOINTS);
  FASTRON_CHECK(chain->a && chain->alpha && chain->d, "chain->a, alpha and d must be non-NULL");
  std::memset(out, 0, sizeof(*out));
  const int n = chain->n;
  out->n = n;
  for (int i = 0; i < n; ++i) {
    double a = chain->a[i], al = chain->alpha[i], d = chain->d[i];
    double th = chain->theta ? chain->theta[i] : 0.0;
    FASTRON_CHECK(std::isfinite(a) && std::isfinite(al) && std::isfinite(d) && std::isfinite(th),
                  "non-finite D-H parameter at joint %d", i);
    int ty = chain->type ? chain->type[i] : 0;
    FASTRON_CHECK(ty == 0 || ty == 1, "joint %d type %d is neither 0 (revolute) nor 1 (prismatic)", i, ty);
    out->a[i] = a;
    out->d[i] = d;
    out->th[i] = th;
    out->ca[i] = std::cos(al);
    out->sa[i] = std::sin(al);
    if (ty == 1) out->prismatic |= 1u << i;
  }
  if (chain->base) {
    const double* b = chain->base;
    for (int k = 0; k < 16; ++k) FASTRON_CHECK(std::isfinite(b[k]), "non-finite base transform entry %d", k);
    FASTRON_CHECK(b[12] == 0.0 && b[13] == 0.0 && b[14] == 0.0 && b[15] == 1.0,
                  "base transform last row must be (0, 0, 0, 1)");
    for (int r = 0; r < 3; ++r) {
      for (int c = 0; c < 3; ++c) out->base_r[3 * r + c] = b[4 * r + c];
      out->base_p[r] = b[4 * r + 3];
    }
  } else {
    out->base_r[0] = out->base_r[4] = out->base_r[8] = 1.0;
  }
  if (!need_points) return FASTRON_OK;
  FASTRON_CHECK(cp != nullptr, "control points are NULL");
  FASTRON_CHECK(cp->M >= 1 && cp->M <= FASTRON_MAX_POINTS, "cp->M = %d outside [1, %d]", cp->M,
                FASTRON_MAX_POINTS);
  FASTRON_CHECK(cp->frame != nullptr, "cp->frame is NULL");
  out->M = cp->M;
  int mm = 0;
  for (int m = 0; m < cp->M; ++m) {
    int f = cp->frame[m];
    FASTRON_CHECK(f >= 0 && f <= n, "control point %d: frame %d outside [0, %d]", m, f, n);
    out->on_frame[f] |= 1u << m;
    for (int k = 0; k < 3; ++k) {
      double o = cp->offset ? cp->offset[3 * m + k] : 0.0;
      FASTRON_CHECK(std::isfinite(o), "non-finite offset of control point %d", m);
      out->off[m][k] = o;
    }
    if (f >= 1) {
      out->slot[m] = mm;
      out->moving[mm++] = m;
    } else {
      out->slot[m] = -1;
    }
  }
  out->Mm = mm;
  // Reach bound: a revolute D-H link moves the next origin by sqrt(a^2 + d^2)
  // whatever its angle; a prismatic one by an unbounded amount. The base
  // matrix B scales lengths by at most sqrt(lambda_max(B^T B)), bounded by the
  // largest absolute row sum of B^T B (Gershgorin; exactly 1 for a rotation).
  double link[FASTRON_MAX_JOINTS + 1];
  link[0] = 0.0;
  for (int i = 0; i < n; ++i)
    link[i + 1] = (out->prismatic >> i & 1u) ? HUGE_VAL : link[i] + std::hypot(out->a[i], out->d[i]);
  double rn = 0.0;
  for (int i = 0; i < 3; ++i) {
    double row = 0.0;
    for (int j = 0; j < 3; ++j) {
      double btb = 0.0;
      for (int k = 0; k < 3; ++k) btb += out->base_r[3 * k + i] * out->base_r[3 * k + j];
      row += std::fabs(btb);
    }
    rn = std::max(rn, row);
  }
  rn = std::sqrt(rn) * (1.0 + 1e-12);
  const double bp = std::sqrt(out->base_p[0] * out->base_p[0] + out->base_p[1] * out->base_p[1] +
                              out->base_p[2] * out->base_p[2]);
  out->reach = 0.0;
  for (int k = 0; k < mm; ++k) {
    const int m = out->moving[k];
    const double off = std::sqrt(out->off[m][0] * out->off[m][0] + out->off[m][1] * out->off[m][1] +
                                 out->off[m][2] * out->off[m][2]);
    out->reach = std::max(out->reach, bp + rn * (link[cp->frame[m]] + off));
  }
  return FASTRON_OK;
}

bool rational_sum_ok(const ChainArgs& c, float gamma, double t_limit) {
  if (c.Mm < 1 || tune_get("score.rational") != 1 || !std::isfinite(c.reach)) return false;
  const double T = 1.01 * (1.0 + 2.0 * (double)gamma * c.reach * c.reach);
  return T <= t_limit && 2.0 * c.Mm * std::log2(T) <= 120.0;
}

// ---------------------------------------------------------------------------
// a1: one thread per configuration.
// ---------------------------------------------------------------------------
// The block's rows of q and of P are contiguous in memory, so both pass
// through LDS: the block reads its 256 n floats and writes its 256 x 3M
// floats with consecutive lanes on consecutive words, and each thread works
// on its own row in LDS. Dynamic LDS: 256 (n + 3M) floats (at most 64 KB).
// Serves chains below 7 joints (FP32 chain); longer chains run
// k_fk_points_fixed below.
// Block copies between global memory and LDS for the FK kernels: 16 bytes per
// lane when both ends are 16-byte aligned (a block's rows start at a multiple
// of 256 rows, so they are whenever the caller's buffer is), else 4.
__device__ __forceinline__ void copy_in(float* __restrict__ dst, const float* __restrict__ src, int count) {
  if ((((uintptr_t)src) & 15) == 0) {
    const int n4 = count >> 2;
    for (int e = threadIdx.x; e < n4; e += 256)
      reinterpret_cast<float4*>(dst)[e] = reinterpret_cast<const float4*>(src)[e];
    for (int e = 4 * n4 + threadIdx.x; e < count; e += 256) dst[e] = src[e];
  } else {
    for (int e = threadIdx.x; e < count; e += 256) dst[e] = src[e];
  }
}
__device__ __forceinline__ void copy_out(float* __restrict__ dst, const float* __restrict__ src, int count) {
  if ((((uintptr_t)dst) & 15) == 0) {
    const int n4 = count >> 2;
    for (int e = threadIdx.x; e < n4; e += 256)
      reinterpret_cast<float4*>(dst)[e] = reinterpret_cast<const float4*>(src)[e];
    for (int e = 4 * n4 + threadIdx.x; e < count; e += 256) dst[e] = src[e];
  } else {
    for (int e = threadIdx.x; e < count; e += 256) dst[e] = src[e];
  }
}

template <typename R>
__global__ void __launch_bounds__(256) k_fk_points(ChainArgs c, const float* __restrict__ q, int64_t N,
                                                    float* __restrict__ P) {
  extern __shared__ float rows[];
  const int n = c.n, w = 3 * c.M;
  float* qs = rows;              // [256][n]
  float* ps = rows + 256 * n;    // [256][w]
  const int64_t j0 = (int64_t)blockIdx.x * 256;
  const int nrow = (int)(N - j0 < 256 ? N - j0 : 256);
  copy_in(qs, q + j0 * n, nrow * n);
  __syncthreads();
  if ((int)threadIdx.x < nrow) {
    float qv[FASTRON_MAX_JOINTS];
#pragma unroll
    for (int i = 0; i < FASTRON_MAX_JOINTS; ++i)
      if (i < n) qv[i] = qs[threadIdx.x * n + i];
    float* out = ps + threadIdx.x * w;
    fk_walk<R>(c, qv, [&](int m, float x, float y, float z) {
      out[3 * m + 0] = x;
      out[3 * m + 1] = y;
      out[3 * m + 2] = z;
    });
  }
  __syncthreads();
  copy_out(P + j0 * w, ps, nrow * w);
}

// ---------------------------------------------------------------------------
// a2: support set -> scoring operands. One thread per (padded) support.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint16_t bf16_rne(float x) {
  uint32_t u = __float_as_uint(x);
  uint32_t r = u + 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(r >> 16);
}
__device__ __forceinline__ float bf16_to_f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// Splits v into `parts` bf16 terms whose sum approximates v (hi, mid, lo).
__device__ __forceinline__ void bf16_split(float v, int parts, uint16_t out[3]) {
  float rem = v;
  for (int k = 0; k < 3; ++k) {
    if (k < parts) {
      out[k] = bf16_rne(rem);
      rem -= bf16_to_f(out[k]);
    } else {
      out[k] = 0;
    }
  }
}

// sum of alpha[s0..s1) by one 256-thread block in a fixed order (strided
// partial sums, then a tree); shared by the single-model and batched forms so
// that both produce the same bits.
__device__ __forceinline__ float block_alpha_sum(const float* __restrict__ alpha, int64_t s0, int64_t s1,
                                                 float* part) {
  float acc = 0.f;
  for (int64_t s = s0 + threadIdx.x; s < s1; s += 256) acc += alpha[s];
  part[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
    __syncthreads();
  }
  return part[0];
}

typedef unsigned short b16row8 __attribute__((ext_vector_type(8)));

// Row `sl` of slot m of a tile's bf16 operand: k = 0..31 stored as [g][s][8]
// (k = 8 g + j), so each group of 8 k values is one 16-byte store.
__device__ __forceinline__ void put_b16_row(uint16_t* __restrict__ B16, int m, int sl, b16row8 g0, b16row8 g1,
                                            b16row8 g2, b16row8 g3) {
  b16row8* row = reinterpret_cast<b16row8*>(B16 + (int64_t)m * 512 + sl * 8);
  row[0] = g0;
  row[16] = g1;
  row[32] = g2;
  row[48] = g3;
}

// Writes one support configuration (or a padding row when sq_row is NULL) as
// row `sl` of its tile T; V (VALU rows) and B16 (bf16 operand of the tile)
// are optional.
template <typename R>
__device__ __forceinline__ void prep_support(const ChainArgs& c, const float* sq_row, float alpha_s, float gamma,
                                             float* __restrict__ T, int sl, int Mp, float* __restrict__ V,
                                             uint16_t* __restrict__ B16) {
  float* A = T;                          // [4][16][Mp]
  float* C = T + tile_c_offset(Mp);      // [4][Mp][4]
  float* W = T + tile_w_offset(Mp);      // [16]
  // defaults: padding and unused slots contribute nothing
  for (int m = 0; m < Mp; ++m) {
    A[(0 * 16 + sl) * Mp + m] = 0.f;
    A[(1 * 16 + sl) * Mp + m] = 0.f;
    A[(2 * 16 + sl) * Mp + m] = 0.f;
    A[(3 * 16 + sl) * Mp + m] = 1.f;
    C[((sl >> 2) * Mp + m) * 4 + (sl & 3)] = 0.f;
    if (V) {
      V[m * 4 + 0] = 0.f; V[m * 4 + 1] = 0.f; V[m * 4 + 2] = 0.f; V[m * 4 + 3] = 0.f;
    }
    // bf16 operand: the unit entries k18-20 (against the parts of the
    // query's norm) are set for padding too, so that a padded row's t is
    // 1 + ||u||^2 >= 1 as in the FP32 layout, never 0
    if (B16) {
      const b16row8 z = {0, 0, 0, 0, 0, 0, 0, 0};
      put_b16_row(B16, m, sl, z, z, (b16row8){0, 0, 0x3f80, 0x3f80, 0x3f80, 0, 0, 0}, z);
    }
  }
  W[sl] = 0.f;
  if (!sq_row) return;
  float qv[FASTRON_MAX_JOINTS];
#pragma unroll
  for (int i = 0; i < FASTRON_MAX_JOINTS; ++i)
    if (i < c.n) qv[i] = sq_row[i];
  const float half_g = 0.5f * gamma;
  fk_walk<R>(c, qv, [&](int m, float x, float y, float z) {
    const int slot = c.slot[m];
    if (slot < 0) return;
    const float ax = -gamma * x, ay = -gamma * y, az = -gamma * z;
    const float cs = half_g * (x * x + y * y + z * z);
    A[(0 * 16 + sl) * Mp + slot] = ax;
    A[(1 * 16 + sl) * Mp + slot] = ay;
    A[(2 * 16 + sl) * Mp + slot] = az;
    C[((sl >> 2) * Mp + slot) * 4 + (sl & 3)] = cs;
    if (V) {
      V[slot * 4 + 0] = ax; V[slot * 4 + 1] = ay; V[slot * 4 + 2] = az; V[slot * 4 + 3] = cs;
    }
    if (B16) {
      // bf16 cross-term operand on the scaled point u' = sqrt(gamma/2) p' (t = 1 + ||u - u'||^2): -2 u'
      // split into hi + mid + lo bf16 terms (exactly -2 times the parts of u'), laid out so that the query
      // side selects the precision: k0-2 hi, k3-5 hi, k6-8 mid, k9-11 hi, k12-14 lo, k15-17 mid, k18-20 = 1,
      // k21-23 the hi/mid/lo parts of ||u'||^2, k24-26 those of ||hi(u')||^2 (the query side puts hi/mid/lo
      // of u against the first six groups, the three parts of its own norm against the ones, and ones
      // against one of the two norms of u': the rounded one for the one-product form, so that its t is that
      // of the rounded points, t >= 1 up to float32 rounding).
      const float sg = sqrtf(half_g);
      const float ux = sg * x, uy = sg * y, uz = sg * z;
      uint16_t sx[3], sy[3], sz[3];
      bf16_split(-2.f * ux, 3, sx);
      bf16_split(-2.f * uy, 3, sy);
      bf16_split(-2.f * uz, 3, sz);
      // both squared norms as explicit fused multiply-adds in the query side's order, so that their
      // rounding does not depend on where the compiler contracts
      uint16_t sc[3], sr[3];
      bf16_split(fmaf(uz, uz, fmaf(uy, uy, ux * ux)), 3, sc);
      const float hx = bf16_to_f(bf16_rne(ux)), hy = bf16_to_f(bf16_rne(uy)), hz = bf16_to_f(bf16_rne(uz));
      bf16_split(fmaf(hz, hz, fmaf(hy, hy, hx * hx)), 3, sr);
      const uint16_t one = 0x3f80;
      put_b16_row(B16, slot, sl,
                  (b16row8){sx[0], sy[0], sz[0], sx[0], sy[0], sz[0], sx[1], sy[1]},   // k0-7
                  (b16row8){sz[1], sx[0], sy[0], sz[0], sx[2], sy[2], sz[2], sx[1]},   // k8-15
                  (b16row8){sy[1], sz[1], one, one, one, sc[0], sc[1], sc[2]},         // k16-23
                  (b16row8){sr[0], sr[1], sr[2], 0, 0, 0, 0, 0});                      // k24-31
    }
  });
  W[sl] = alpha_s / (float)c.M;
}

template <typename R>
__global__ void __launch_bounds__(256) k_support_prep(ChainArgs c, const float* __restrict__ sq,
                                                       const float* __restrict__ alpha, int64_t S, int64_t ntiles,
                                                       float gamma, float fixed_scale, char* __restrict__ blob) {
  if (blockIdx.x == 0) {
    // header: f_const = fixed_scale * sum_i alpha_i (the folded base-frame points), the rest zero
    __shared__ float part[256];
    const float fc = fixed_scale != 0.f ? block_alpha_sum(alpha, 0, S, part) * fixed_scale : 0.f;
    if (threadIdx.x < kHeaderBytes / 4) reinterpret_cast<float*>(blob)[threadIdx.x] = threadIdx.x == 0 ? fc : 0.f;
  }
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= ntiles * kTile) return;
  const int Mp = (c.M + 3) & ~3;
  const int64_t tile = s / kTile;
  const int sl = (int)(s % kTile);
  float* T = reinterpret_cast<float*>(blob + kHeaderBytes) + tile * tile_floats(Mp);
  const int64_t S_pad = ntiles * kTile;
  float* V = reinterpret_cast<float*>(blob + kHeaderBytes + ntiles * tile_floats(Mp) * 4) + s * Mp * 4;
  uint16_t* B16 = reinterpret_cast<uint16_t*>(blob + kHeaderBytes + ntiles * tile_floats(Mp) * 4 +
                                              S_pad * Mp * 4 * 4) +
                  tile * (int64_t)Mp * 512;
  const bool real = s < S;
  prep_support<R>(c, real ? sq + s * c.n : nullptr, real ? alpha[s] : 0.f, gamma, T, sl, Mp, V, B16);
}

// Batched form: E support sets concatenated (support_off[E + 1]), each padded
// to whole tiles (tile_off[E + 1]); FP32 tiles only. One thread per padded row.
template <typename R>
__global__ void __launch_bounds__(256) k_support_prep_batched(ChainArgs c, const float* __restrict__ sq,
                                                               const float* __restrict__ alpha,
                                                               const int64_t* __restrict__ support_off,
                                                               const int64_t* __restrict__ tile_off, int E,
                                                               float gamma, float* __restrict__ tiles) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t total_tiles = tile_off[E];
  if (p >= total_tiles * kTile) return;
  const int Mp = (c.M + 3) & ~3;
  const int64_t tile = p / kTile;
  const int sl = (int)(p % kTile);
  int lo = 0, hi = E;  // largest e with tile_off[e] <= tile
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (tile_off[mid] <= tile) lo = mid; else hi = mid;
  }
  const int64_t s = support_off[lo] + (tile - tile_off[lo]) * kTile + sl;
  const bool real = s < support_off[lo + 1];
  prep_support<R>(c, real ? sq + s * c.n : nullptr, real ? alpha[s] : 0.f, gamma,
                  tiles + tile * tile_floats(Mp), sl, Mp, nullptr, nullptr);
}


// Per-environment fixed-point term: one block per environment.
__global__ void __launch_bounds__(256) k_fixed_term_batched(const float* __restrict__ alpha,
                                                            const int64_t* __restrict__ support_off, float scale,
                                                            float* __restrict__ f_const) {
  __shared__ float part[256];
  const int e = blockIdx.x;
  const float sum = block_alpha_sum(alpha, support_off[e], support_off[e + 1], part);
  if (threadIdx.x == 0) f_const[e] = sum * scale;
}

fastron_status launch_prep_batched(const ChainArgs& c, const float* sq, const float* alpha,
                                   const int64_t* support_off_d, const int64_t* tile_off_d, int E,
                                   int64_t total_tiles, float gamma, float* tiles, float* f_const, hipStream_t s) {
  if (total_tiles > 0) {
    const unsigned blocks = (unsigned)((total_tiles * kTile + 255) / 256);
    if (c.n >= kFp64Joints)
      hipLaunchKernelGGL(k_support_prep_batched<double>, dim3(blocks), dim3(256), 0, s, c, sq, alpha, support_off_d,
                         tile_off_d, E, gamma, tiles);
    else
      hipLaunchKernelGGL(k_support_prep_batched<float>, dim3(blocks), dim3(256), 0, s, c, sq, alpha, support_off_d,
                         tile_off_d, E, gamma, tiles);
    FASTRON_HIP(hipGetLastError());
  }
  const float scale = (float)(c.M - c.Mm) / (float)c.M;
  hipLaunchKernelGGL(k_fixed_term_batched, dim3((unsigned)E), dim3(256), 0, s, alpha, support_off_d, scale, f_const);
  FASTRON_HIP(hipGetLastError());
  return FASTRON_OK;
}

// f_const = (#fixed points / M) * sum_s alpha_s.

__global__ void k_zero_header(float* header) {
  if (threadIdx.x < 64) header[threadIdx.x] = 0.f;
}

// FP64 sine and cosine without branches for |x| <= kSinCosReduceMax: Cody and
// Waite's reduction by pi/2 (the quadrant k = rint(2x/pi) and
// r = x - k pi/2 with pi/2 split into three doubles, each product applied by
// one fused multiply-add), then the Taylor polynomials of sin and cos on
// |r| <= pi/4 through degree 17 and 16, and the quadrant's signs and swap.
// Measured against long double over 4e7 arguments up to |x| = 1e5: at most
// 1.2 units of 2^-53 absolute error. Larger arguments take the library
// routine.
constexpr double kSinCosReduceMax = 1e5;

__device__ __forceinline__ void sincos_reduced(double x, double* s, double* c) {
  const double k = rint(x * 0.63661977236758134308);  // 2/pi
  double r = fma(-k, 1.5707963267948966, x);
  r = fma(-k, 6.123233995736766e-17, r);
  r = fma(-k, -1.4973849048591698e-33, r);
  const double z = r * r;
  double p = 1.0 / 355687428096000.0;  // 1/17!
  p = fma(p, z, -1.0 / 1307674368000.0);
  p = fma(p, z, 1.0 / 6227020800.0);
  p = fma(p, z, -1.0 / 39916800.0);
  p = fma(p, z, 1.0 / 362880.0);
  p = fma(p, z, -1.0 / 5040.0);
  p = fma(p, z, 1.0 / 120.0);
  p = fma(p, z, -1.0 / 6.0);
  const double sn = fma(r * z, p, r);
  double t = 1.0 / 20922789888000.0;  // 1/16!
  t = fma(t, z, -1.0 / 87178291200.0);
  t = fma(t, z, 1.0 / 479001600.0);
  t = fma(t, z, -1.0 / 3628800.0);
  t = fma(t, z, 1.0 / 40320.0);
  t = fma(t, z, -1.0 / 720.0);
  t = fma(t, z, 1.0 / 24.0);
  t = fma(t, z, -0.5);
  const double cs = fma(z, t, 1.0);
  const int quad = (int)(int64_t)k & 3;
  const double ss = (quad & 1) ? cs : sn, cc = (quad & 1) ? sn : cs;
  *s = (quad & 2) ? -ss : ss;
  *c = ((quad + 1) & 2) ? -cc : cc;
}

// FP64 chains of exactly NJ joints: every joint's sine and cosine first, as
// straight-line code the compiler can interleave (they are independent of
// one another), then the chain product of Eq. 1 with the control points of
// Eq. 2 written as they are reached. Same staging of q and P through LDS as
// k_fk_points. (Storing each row of P straight from registers measured 0.26
// against 0.18 ms on 4,194,304 7-joint configurations, and padding the LDS
// rows to an odd stride 0.21 ms.)
template <int NJ>
__global__ void __launch_bounds__(256) k_fk_points_fixed(ChainArgs c, const float* __restrict__ q, int64_t N,
                                                          float* __restrict__ P) {
  extern __shared__ float rows[];
  const int w = 3 * c.M;
  float* qs = rows;              // [256][NJ]
  float* ps = rows + 256 * NJ;   // [256][w]
  const int64_t j0 = (int64_t)blockIdx.x * 256;
  const int nrow = (int)(N - j0 < 256 ? N - j0 : 256);
  copy_in(qs, q + j0 * NJ, nrow * NJ);
  __syncthreads();
  if ((int)threadIdx.x < nrow) {
    double st[NJ], ct[NJ], dd[NJ];
    bool wide = false;
#pragma unroll
    for (int i = 0; i < NJ; ++i) {
      const double qi = (double)qs[threadIdx.x * NJ + i];
      const bool pr = (c.prismatic >> i) & 1u;
      const double th = c.th[i] + (pr ? 0.0 : qi);
      dd[i] = c.d[i] + (pr ? qi : 0.0);
      sincos_reduced(th, &st[i], &ct[i]);
      wide |= !(fabs(th) <= kSinCosReduceMax);
    }
    if (wide) {
#pragma unroll
      for (int i = 0; i < NJ; ++i) {
        const double qi = (double)qs[threadIdx.x * NJ + i];
        const double th = c.th[i] + (((c.prismatic >> i) & 1u) ? 0.0 : qi);
        if (!(fabs(th) <= kSinCosReduceMax)) sincos(th, &st[i], &ct[i]);
      }
    }
    float* out = ps + threadIdx.x * w;
    double xx = c.base_r[0], xy = c.base_r[3], xz = c.base_r[6];
    double yx = c.base_r[1], yy = c.base_r[4], yz = c.base_r[7];
    double zx = c.base_r[2], zy = c.base_r[5], zz = c.base_r[8];
    double px = c.base_p[0], py = c.base_p[1], pz = c.base_p[2];
    auto emit_frame = [&](int fi) {
      uint32_t mask = c.on_frame[fi];
      while (mask) {
        const int m = __builtin_ctz(mask);
        mask &= mask - 1;
        const double ox = c.off[m][0], oy = c.off[m][1], oz = c.off[m][2];
        out[3 * m + 0] = (float)(px + ox * xx + oy * yx + oz * zx);
        out[3 * m + 1] = (float)(py + ox * xy + oy * yy + oz * zy);
        out[3 * m + 2] = (float)(pz + ox * xz + oy * yz + oz * zz);
      }
    };
    emit_frame(0);
#pragma unroll
    for (int i = 0; i < NJ; ++i) {
      const double sv = st[i], cv = ct[i];
      const double ux = cv * xx + sv * yx, uy = cv * xy + sv * yy, uz = cv * xz + sv * yz;
      const double vx = cv * yx - sv * xx, vy = cv * yy - sv * xy, vz = cv * yz - sv * xz;
      const double a = c.a[i], cal = c.ca[i], sal = c.sa[i];
      px += a * ux + dd[i] * zx;
      py += a * uy + dd[i] * zy;
      pz += a * uz + dd[i] * zz;
      xx = ux; xy = uy; xz = uz;
      const double nzx = cal * zx - sal * vx, nzy = cal * zy - sal * vy, nzz = cal * zz - sal * vz;
      yx = cal * vx + sal * zx; yy = cal * vy + sal * zy; yz = cal * vz + sal * zz;
      zx = nzx; zy = nzy; zz = nzz;
      emit_frame(i + 1);
    }
  }
  __syncthreads();
  copy_out(P + j0 * w, ps, nrow * w);
}

}  // namespace fastron

using namespace fastron;

extern "C" {

const char* fastron_last_error(void) { return g_err; }

const char* fastron_version(void) { return "fastron-fk gfx950 1.0"; }

fastron_status fastron_control_point_frames(const fastron_chain* chain, int32_t include_base, int32_t* frame,
                                           int32_t* M) {
  clear_error();
  FASTRON_CHECK(chain != nullptr && frame != nullptr && M != nullptr, "chain, frame and M must be non-NULL");
  FASTRON_CHECK(chain->n >= 1 && chain->n <= FASTRON_MAX_JOINTS, "chain->n = %d outside [1, %d]", chain->n,
                FASTRON_MAX_JOINTS);
  FASTRON_CHECK(chain->a && chain->d, "chain->a and d must be non-NULL");
  int32_t count = 0;
  if (include_base) frame[count++] = 0;
  for (int32_t i = 1; i <= chain->n; ++i) {
    const bool prismatic = chain->type && chain->type[i - 1] == 1;
    // a revolute joint with no link length and no offset keeps the preceding origin
    if (!prismatic && chain->a[i - 1] == 0.0 && chain->d[i - 1] == 0.0) continue;
    frame[count++] = i;
  }
  *M = count;
  return FASTRON_OK;
}

int64_t fastron_model_bytes(int64_t S, int32_t M) {
  if (S < 0 || M < 1 || M > FASTRON_MAX_POINTS) return -1;
  return model_bytes(S, M);
}

fastron_status fastron_fk_points(const fastron_chain* chain, const fastron_cpoints* cp, const float* q, int64_t N,
                                 float* P, void* stream) {
  clear_error();
  ChainArgs c;
  fastron_status st = pack_chain(chain, cp, &c, true);
  if (st != FASTRON_OK) return st;
  FASTRON_CHECK(N >= 0, "N = %lld < 0", (long long)N);
  if (N == 0) return FASTRON_OK;
  FASTRON_CHECK(q && P, "q and P must be non-NULL");
  FASTRON_CHECK(aligned(q, 4) && aligned(P, 4), "q and P must be 4-byte aligned");
  const int64_t blocks = (N + 255) / 256;
  FASTRON_CHECK(grid_fits(blocks, 256), "N = %lld above one launch's 2^32 - 256 configurations", (long long)N);
  const size_t lds = (size_t)256 * (c.n + 3 * c.M) * sizeof(float);
  const dim3 grid((unsigned)blocks);
  hipStream_t s = as_stream(stream);
#define FASTRON_FK_FIXED(K) \
  case K: hipLaunchKernelGGL(k_fk_points_fixed<K>, grid, dim3(256), lds, s, c, q, N, P); break;
  if (c.n >= kFp64Joints) {
    switch (c.n) {
      FASTRON_FK_FIXED(7) FASTRON_FK_FIXED(8) FASTRON_FK_FIXED(9) FASTRON_FK_FIXED(10) FASTRON_FK_FIXED(11)
      FASTRON_FK_FIXED(12) FASTRON_FK_FIXED(13) FASTRON_FK_FIXED(14) FASTRON_FK_FIXED(15) FASTRON_FK_FIXED(16)
      default: return fail(FASTRON_EINVAL, "n = %d joints outside [7, 16]", c.n);  // pack_chain bounds n
    }
  } else
    hipLaunchKernelGGL(k_fk_points<float>, grid, dim3(256), lds, s, c, q, N, P);
#undef FASTRON_FK_FIXED
  FASTRON_HIP(hipGetLastError());
  return FASTRON_OK;
}

fastron_status fastron_support_prep(const fastron_chain* chain, const fastron_cpoints* cp, const float* support_q,
                                    const float* alpha, int64_t S, float gamma, fastron_model* model, void* stream) {
  clear_error();
  ChainArgs c;
  fastron_status st = pack_chain(chain, cp, &c, true);
  if (st != FASTRON_OK) return st;
  FASTRON_CHECK(model != nullptr, "model is NULL");
  FASTRON_CHECK(S >= 0, "S = %lld < 0", (long long)S);
  FASTRON_CHECK(std::isfinite(gamma) && gamma > 0.f, "gamma must be finite and > 0");
  FASTRON_CHECK(model->data != nullptr, "model->data is NULL");
  FASTRON_CHECK(aligned(model->data, 256), "model->data must be 256-byte aligned");
  const int64_t need = model_bytes(S, c.M);
  FASTRON_CHECK(model->bytes >= need, "model->bytes = %lld < %lld needed", (long long)model->bytes,
                (long long)need);
  FASTRON_CHECK(S == 0 || (support_q && alpha), "support_q and alpha must be non-NULL when S > 0");
  model->S = S;
  model->M = c.M;
  model->gamma = gamma;
  hipStream_t s = as_stream(stream);
  char* blob = static_cast<char*>(model->data);
  const int64_t nt = ntiles_of(S);
  if (nt == 0) {
    hipLaunchKernelGGL(k_zero_header, dim3(1), dim3(64), 0, s, reinterpret_cast<float*>(blob));
  } else {
    // one launch: the tiles, and in block 0 the header with the folded base-frame term
    const float fixed_scale = c.Mm < c.M ? (float)(c.M - c.Mm) / (float)c.M : 0.f;
    const int64_t threads = nt * kTile;
    const unsigned blocks = (unsigned)((threads + 255) / 256);
    if (c.n >= kFp64Joints)
      hipLaunchKernelGGL(k_support_prep<double>, dim3(blocks), dim3(256), 0, s, c, support_q, alpha, S, nt, gamma,
                         fixed_scale, blob);
    else
      hipLaunchKernelGGL(k_support_prep<float>, dim3(blocks), dim3(256), 0, s, c, support_q, alpha, S, nt, gamma,
                         fixed_scale, blob);
  }
  FASTRON_HIP(hipGetLastError());
  return FASTRON_OK;
}

}  // extern "C"
