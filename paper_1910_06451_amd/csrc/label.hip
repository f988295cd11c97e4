// Geometric labels for training and evaluation data. Stands in for the
// ground-truth collision checker of Section IV (the paper labels with FCL on
// robot meshes, which is not available here): link i of the arm is a capsule
// of radius r around the segment between the origins of frames i-1 and i,
// obstacles are axis-aligned boxes, and a configuration is in collision (+1)
// when some capsule touches some box.
//
// Segment-to-box distance: with P(t) = A + t (B - A), the squared distance
// g(t) = sum_k e_k(t)^2, e_k = max(lo_k - P_k, 0, P_k - hi_k), is convex and
// continuously differentiable on [0, 1], so its derivative
// g'(t) = 2 sum_k s_k e_k(t) (B_k - A_k) is non-decreasing. The minimiser is
// t = 0 if g'(0) >= 0, t = 1 if g'(1) <= 0, and otherwise the root of g',
// found here by bisection to double-precision resolution. Everything is FP64,
// one thread per configuration.
//
// Culling: the gap between the box and the segment's bounding box is a lower
// bound on their distance, so a (link, box) pair whose gap exceeds the best
// distance found so far (plus 1e-12 m, far above the rounding of either
// computation) cannot lower the minimum and is skipped. When only labels are
// asked for, a configuration stops at its first touching pair.
#include <cmath>

#include "fastron_internal.h"

namespace fastron {

__device__ __forceinline__ double excess(double u, double lo, double hi, double* sgn) {
  if (u < lo) {
    *sgn = -1.0;
    return lo - u;
  }
  if (u > hi) {
    *sgn = 1.0;
    return u - hi;
  }
  *sgn = 0.0;
  return 0.0;
}

__device__ __forceinline__ double seg_box_d2(const double A[3], const double D[3], const double* box) {
  auto g_and_dg = [&](double t, double* dg) {
    double g = 0.0, d = 0.0;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      double sgn;
      const double e = excess(A[k] + t * D[k], box[k], box[3 + k], &sgn);
      g += e * e;
      d += 2.0 * sgn * e * D[k];
    }
    *dg = d;
    return g;
  };
  double d0, d1;
  const double g0 = g_and_dg(0.0, &d0);
  if (d0 >= 0.0) return g0;
  const double g1 = g_and_dg(1.0, &d1);
  if (d1 <= 0.0) return g1;
  double lo = 0.0, hi = 1.0;
  for (int it = 0; it < 64; ++it) {
    const double mid = 0.5 * (lo + hi);
    if (mid <= lo || mid >= hi) break;
    double dm;
    g_and_dg(mid, &dm);
    if (dm < 0.0) lo = mid; else hi = mid;
  }
  double dl, dh;
  const double gl = g_and_dg(lo, &dl), gh = g_and_dg(hi, &dh);
  return fmin(gl, gh);
}

// Squared gap between the box and the bounding box of the segment A -> A + D.
__device__ __forceinline__ double bbox_gap2(const double A[3], const double D[3], const double* box) {
  double s = 0.0;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const double b = A[k] + D[k];
    const double g = fmax(fmax(box[k] - fmax(A[k], b), fmin(A[k], b) - box[3 + k]), 0.0);
    s += g * g;
  }
  return s;
}

__global__ void __launch_bounds__(256) k_label(ChainArgs c, const float* __restrict__ q, int64_t N, double radius,
                                                const double* __restrict__ boxes, int nbox,
                                                int8_t* __restrict__ label, float* __restrict__ clearance) {
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (j >= N) return;
  // frame origins: walk the chain in FP64 (Section II-A, Eq. 1)
  double xx = c.base_r[0], xy = c.base_r[3], xz = c.base_r[6];
  double yx = c.base_r[1], yy = c.base_r[4], yz = c.base_r[7];
  double zx = c.base_r[2], zy = c.base_r[5], zz = c.base_r[8];
  double o[3] = {c.base_p[0], c.base_p[1], c.base_p[2]};
  double best = INFINITY;
  for (int i = 0; i < c.n; ++i) {
    const double qi = (double)q[j * c.n + i];
    double th = c.th[i], dd = c.d[i];
    if ((c.prismatic >> i) & 1u) dd += qi; else th += qi;
    double st, ct;
    sincos(th, &st, &ct);
    const double ux = ct * xx + st * yx, uy = ct * xy + st * yy, uz = ct * xz + st * yz;
    const double vx = ct * yx - st * xx, vy = ct * yy - st * xy, vz = ct * yz - st * xz;
    const double a = c.a[i], cal = c.ca[i], sal = c.sa[i];
    const double A[3] = {o[0], o[1], o[2]};
    o[0] += a * ux + dd * zx;
    o[1] += a * uy + dd * zy;
    o[2] += a * uz + dd * zz;
    xx = ux; xy = uy; xz = uz;
    const double nzx = cal * zx - sal * vx, nzy = cal * zy - sal * vy, nzz = cal * zz - sal * vz;
    yx = cal * vx + sal * zx; yy = cal * vy + sal * zy; yz = cal * vz + sal * zz;
    zx = nzx; zy = nzy; zz = nzz;
    const double D[3] = {o[0] - A[0], o[1] - A[1], o[2] - A[2]};
    for (int b = 0; b < nbox; ++b) {
      const double reach = best + radius + 1e-12;  // >= 1e-12: best >= -radius
      if (bbox_gap2(A, D, boxes + 6 * b) > reach * reach) continue;
      const double d = sqrt(seg_box_d2(A, D, boxes + 6 * b)) - radius;
      best = fmin(best, d);
    }
    if (!clearance && best <= 0.0) break;
  }
  label[j] = (best <= 0.0) ? (int8_t)1 : (int8_t)-1;
  if (clearance) clearance[j] = (float)best;
}

}  // namespace fastron

using namespace fastron;

extern "C" fastron_status fastron_label_capsule_box(const fastron_chain* chain, const float* q, int64_t N,
                                                    double radius, const double* boxes, int32_t nbox, int8_t* label,
                                                    float* clearance, void* stream) {
  clear_error();
  ChainArgs c;
  fastron_status st = pack_chain(chain, nullptr, &c, false);
  if (st != FASTRON_OK) return st;
  FASTRON_CHECK(N >= 0, "N < 0");
  FASTRON_CHECK(std::isfinite(radius) && radius >= 0.0, "radius must be finite and >= 0");
  FASTRON_CHECK(nbox >= 0 && nbox <= 4096, "nbox = %d outside [0, 4096]", nbox);
  if (N == 0) return FASTRON_OK;
  FASTRON_CHECK(q && label, "q and label must be non-NULL");
  FASTRON_CHECK(nbox == 0 || boxes != nullptr, "boxes is NULL");
  const int64_t blocks = (N + 255) / 256;
  FASTRON_CHECK(grid_fits(blocks, 256), "N = %lld above one launch's 2^32 - 256 configurations", (long long)N);
  hipLaunchKernelGGL(k_label, dim3((unsigned)blocks), dim3(256), 0, as_stream(stream), c, q, N, radius, boxes, nbox,
                     label, clearance);
  FASTRON_HIP(hipGetLastError());
  return FASTRON_OK;
}
