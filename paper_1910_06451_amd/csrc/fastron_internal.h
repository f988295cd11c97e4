// Internal definitions shared by the library's translation units (host
// validation, error reporting, kernel-argument packing and the device-side
// forward kinematics). Not installed; the public ABI is include/fastron_fk.h.
#pragma once

#include <type_traits>

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdint>
#include <cstdio>

#include "fastron_fk.h"

namespace fastron {

// ---------------------------------------------------------------------------
// Errors: a thread-local message plus a status code. Every entry point calls
// clear_error() first, validates on the host, and only then touches HIP.
// ---------------------------------------------------------------------------
void clear_error();
fastron_status fail(fastron_status st, const char* fmt, ...) __attribute__((format(printf, 2, 3)));

#define FASTRON_HIP(expr)                                                                     \
  do {                                                                                        \
    hipError_t e_ = (expr);                                                                   \
    if (e_ != hipSuccess)                                                                     \
      return ::fastron::fail(e_ == hipErrorOutOfMemory ? FASTRON_ENOMEM : FASTRON_EHIP,       \
                             "%s failed: %s", #expr, hipGetErrorString(e_));                  \
  } while (0)

#define FASTRON_CHECK(cond, ...)                                     \
  do {                                                               \
    if (!(cond)) return ::fastron::fail(FASTRON_EINVAL, __VA_ARGS__); \
  } while (0)

// ---------------------------------------------------------------------------
// Chain + control points as a by-value kernel argument. Kernel arguments sit
// in the constant kernarg segment and are read with scalar loads, so every
// D-H parameter is a wave-uniform constant inside the kernels.
// ---------------------------------------------------------------------------
struct ChainArgs {
  int32_t n;          // joints
  int32_t M;          // control points
  int32_t Mm;         // control points that move (frame >= 1)
  uint32_t prismatic; // bit i set: joint i is prismatic
  double a[FASTRON_MAX_JOINTS];
  double d[FASTRON_MAX_JOINTS];
  double th[FASTRON_MAX_JOINTS];
  double ca[FASTRON_MAX_JOINTS];  // cos(alpha_i)
  double sa[FASTRON_MAX_JOINTS];  // sin(alpha_i)
  double base_r[9];               // base rotation, row-major
  double base_p[3];               // base translation
  double off[FASTRON_MAX_POINTS][3];
  uint32_t on_frame[FASTRON_MAX_JOINTS + 1];  // bit m set: control point m sits on frame i
  int32_t moving[FASTRON_MAX_POINTS];         // indices of the moving control points, in order
  int32_t slot[FASTRON_MAX_POINTS];           // rank of point m among the moving points, -1 if fixed
  double reach;  // upper bound on |p| over the moving points and all joint values (inf past a prismatic joint)
};

// Validates chain and control points and packs them. `need_points` = false
// for entry points that only use the chain (the labeller).
fastron_status pack_chain(const fastron_chain* chain, const fastron_cpoints* cp, ChainArgs* out, bool need_points);

// Whether the scoring kernels may sum 1/t^2 over a pair's control points as
// one running fraction (no per-value reciprocal, no saturation): true when
// the chain's reach bound R caps t = 1 + gamma/2 ||p - p'||^2 at
// T = 1 + 2 gamma R^2 (with 1 % slack) such that T^(2 Mm) <= 2^120, so the
// fraction's denominator and numerator stay finite and normal, and
// T <= t_limit, so that t's own rounding error keeps it far from 0 without
// the saturation: 2^16 where t is formed to FP32 accuracy (error a few units
// of 2^-24 times T), 2^8 for one bf16 product per coordinate (error about
// 2^-8 gamma R^2). The tuning key score.rational = 0 switches the form off.
bool rational_sum_ok(const ChainArgs& c, float gamma, double t_limit = 65536.0);

// Tuning table lookup (-1 for an unknown key).
int64_t tune_get(const char* key);

// Stream helper.
inline hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

// Device pointer sanity (host check only: non-null and aligned).
inline bool aligned(const void* p, size_t a) { return (reinterpret_cast<uintptr_t>(p) % a) == 0; }

// A dispatch spans at most 2^32 - 1 work-items per grid dimension (the
// dispatch packet holds the grid size in 32 bits): `blocks` workgroups of
// `threads` work-items fit if their product does.
inline bool grid_fits(int64_t blocks, int threads) { return blocks >= 0 && blocks <= (int64_t)UINT32_MAX / threads; }

// ---------------------------------------------------------------------------
// Device-side forward kinematics (Section II-A, Eq. 1 and Eq. 2).
//
// The chain is walked frame by frame, keeping the frame's axes (columns of
// the rotation) and origin. Appending link i with angle th, twist al, length
// a and offset d (Eq. 1) gives, with u = c(th) x + s(th) y and
// v = -s(th) x + c(th) y:
//   origin' = origin + a u + d z,   x' = u,   y' = c(al) v + s(al) z,
//   z' = -s(al) v + c(al) z
// which is the product wA_{i-1} (i-1)A_i written column by column. Control
// point m on frame j is origin_j + R_j offset_m (Eq. 2 with T_m a
// translation). `emit(m, x, y, z)` receives each point as float.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void sincos_r(double x, double* s, double* c) { sincos(x, s, c); }
__device__ __forceinline__ void sincos_r(float x, float* s, float* c) { sincosf(x, s, c); }

// Hardware sine / cosine (absolute error about 1e-6 for the joint ranges
// here): for consumers that round the positions far more coarsely right
// after, such as the screening network's BF16 features.
struct FastTrig {};
__device__ __forceinline__ void sincos_r(float x, float* s, float* c, FastTrig) {
  *s = __sinf(x);
  *c = __cosf(x);
}

// R = double or float; R = FastTrig computes in float with hardware sin/cos.
template <typename R>
struct FkReal {
  typedef R type;
};
template <>
struct FkReal<FastTrig> {
  typedef float type;
};

template <typename RT, typename Emit>
__device__ __forceinline__ void fk_walk(const ChainArgs& c, const float* q, Emit&& emit) {
  typedef typename FkReal<RT>::type R;
  R xx = (R)c.base_r[0], xy = (R)c.base_r[3], xz = (R)c.base_r[6];
  R yx = (R)c.base_r[1], yy = (R)c.base_r[4], yz = (R)c.base_r[7];
  R zx = (R)c.base_r[2], zy = (R)c.base_r[5], zz = (R)c.base_r[8];
  R px = (R)c.base_p[0], py = (R)c.base_p[1], pz = (R)c.base_p[2];
  auto emit_frame = [&](int fi) {
    uint32_t mask = c.on_frame[fi];
    while (mask) {
      int m = __builtin_ctz(mask);
      mask &= mask - 1;
      R ox = (R)c.off[m][0], oy = (R)c.off[m][1], oz = (R)c.off[m][2];
      R X = px + ox * xx + oy * yx + oz * zx;
      R Y = py + ox * xy + oy * yy + oz * zy;
      R Z = pz + ox * xz + oy * yz + oz * zz;
      emit(m, (float)X, (float)Y, (float)Z);
    }
  };
  emit_frame(0);
  for (int i = 0; i < c.n; ++i) {
    R qi = (R)q[i];
    R th = (R)c.th[i], dd = (R)c.d[i];
    if ((c.prismatic >> i) & 1u) dd += qi; else th += qi;
    R st, ct;
    if constexpr (std::is_same<RT, FastTrig>::value)
      sincos_r(th, &st, &ct, FastTrig{});
    else
      sincos_r(th, &st, &ct);
    R ux = ct * xx + st * yx, uy = ct * xy + st * yy, uz = ct * xz + st * yz;
    R vx = ct * yx - st * xx, vy = ct * yy - st * xy, vz = ct * yz - st * xz;
    R a = (R)c.a[i], cal = (R)c.ca[i], sal = (R)c.sa[i];
    px += a * ux + dd * zx;
    py += a * uy + dd * zy;
    pz += a * uz + dd * zz;
    xx = ux; xy = uy; xz = uz;
    R nzx = cal * zx - sal * vx, nzy = cal * zy - sal * vy, nzz = cal * zz - sal * vz;
    yx = cal * vx + sal * zx; yy = cal * vy + sal * zy; yz = cal * vz + sal * zz;
    zx = nzx; zy = nzy; zz = nzz;
    emit_frame(i + 1);
  }
}

// Batched support preparation (fk.hip): FP32 tiles of E support sets and the
// per-environment fixed-point terms.
fastron_status launch_prep_batched(const ChainArgs& c, const float* sq, const float* alpha,
                                   const int64_t* support_off_d, const int64_t* tile_off_d, int E,
                                   int64_t total_tiles, float gamma, float* tiles, float* f_const, hipStream_t s);

// Threshold from which the chain product runs in FP64.
constexpr int kFp64Joints = 7;

}  // namespace fastron
