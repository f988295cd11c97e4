// Gram columns and the Fastron model update (Section III-B, Eq. 5-9 and
// Algorithm 1) on the device.
//
// fastron_gram_update: one thread per training point j evaluates
//   K_FK(X_j, X_i) = (1/M) sum_m (1 + gamma/2 ||FK_m(X_j) - FK_m(X_i)||^2)^-2
// with direct differences (HBM-bound: 12M bytes of control points per j) and
// applies F_j += dalpha * K_ji.
//
// fastron_train: Algorithm 1 is strictly sequential -- every iteration needs
// the global argmin of the margins before the next column can be chosen -- so
// it runs as ONE persistent, cooperatively launched grid. Each workgroup owns
// a contiguous slice of the training set. Per iteration each workgroup:
//   1. publishes one record for its slice (min margin and its index, the
//      weight at that index, max of y(F - alpha) over alpha != 0 and its
//      index and weight, and its count of nonzero weights), every word tagged
//      with the low byte of the iteration number;
//   2. waits until it has read every workgroup's record of this iteration
//      (no central barrier: a record is complete when all its words carry the
//      current tag);
//   3. reduces all records itself (identically in every workgroup, so every
//      workgroup takes the same decision without a second exchange);
//   4. applies the add or the removal to its slice in one pass that also
//      builds its next record.
// Records are double-buffered by iteration parity. The wait is bounded by a
// constant-clock budget and reports FASTRON_EDEVICE instead of hanging.
#include <cmath>
#include <vector>

#include "fastron_internal.h"

namespace fastron {

// ---------------------------------------------------------------------------
// a4: Gram column + F update
// ---------------------------------------------------------------------------
// ---------------------------------------------------------------------------
// a5: persistent Algorithm 1
// ---------------------------------------------------------------------------
template <typename T>
struct Rec {
  T minval;       // min over the slice of y_j F_j
  T a_at_min;     // alpha at that index
  T maxval;       // max over the slice of y_j (F_j - alpha_j), alpha_j != 0
  T a_at_max;     // alpha at that index
  int32_t minidx; // -1 if the slice is empty
  int32_t maxidx; // -1 if no nonzero weight in the slice
  int32_t count;  // number of nonzero weights in the slice
  int32_t ymin;   // label y at minidx (so the decision needs no lookup)
};

template <typename T>
struct TrainState {
  const float* P;
  const int8_t* y;
  T* alpha;
  T* F;
  Rec<T>* rec;         // record words [2][G][K]
  int64_t* out;        // [0] updates, [1] status (0 break, 1 iter_max, -5 exchange timeout)
  int32_t* trace_act;
  int32_t* trace_idx;
  int64_t trace_cap;
  int64_t N;
  int64_t iter_max;
  int64_t s_max;
  T half_g;
  T beta;
  int M;
  int D;               // coordinates per point: 3 for control points, n for joint vectors
  int chunk;           // training points per workgroup
  long long timeout;    // wait limit for the record exchange, in constant-clock ticks
  int poll_delay;       // wave form: sleeps (64 clocks each) before the first poll; -1 = adaptive
  int p_in_lds;         // the slice's control points are staged in LDS
  // several independent training sets in one launch (wave form only):
  // workgroup w trains set env_of[w], whose workgroups are env_wg0[e] ..
  // env_wg0[e + 1] - 1, whose points are env_off[e] .. env_off[e + 1] - 1, and
  // whose (updates, status) go to out[2 e], out[2 e + 1]. NULL: one set.
  const int32_t* env_of;
  const int32_t* env_wg0;
  const int64_t* env_off;
};

template <typename T>
__device__ __forceinline__ void rec_merge(Rec<T>& a, const Rec<T>& b) {
  if (b.minidx >= 0 && (a.minidx < 0 || b.minval < a.minval || (b.minval == a.minval && b.minidx < a.minidx))) {
    a.minval = b.minval;
    a.a_at_min = b.a_at_min;
    a.minidx = b.minidx;
    a.ymin = b.ymin;
  }
  if (b.maxidx >= 0 && (a.maxidx < 0 || b.maxval > a.maxval || (b.maxval == a.maxval && b.maxidx < a.maxidx))) {
    a.maxval = b.maxval;
    a.a_at_max = b.a_at_max;
    a.maxidx = b.maxidx;
  }
  a.count += b.count;
}

template <typename T>
__device__ __forceinline__ Rec<T> rec_empty() {
  Rec<T> r;
  r.minval = 0;
  r.a_at_min = 0;
  r.maxval = 0;
  r.a_at_max = 0;
  r.minidx = -1;
  r.maxidx = -1;
  r.count = 0;
  r.ymin = 0;
  return r;
}

template <typename T>
__device__ __forceinline__ Rec<T> rec_shfl_down(const Rec<T>& r, int off) {
  Rec<T> o;
  o.minval = __shfl_down(r.minval, off);
  o.a_at_min = __shfl_down(r.a_at_min, off);
  o.maxval = __shfl_down(r.maxval, off);
  o.a_at_max = __shfl_down(r.a_at_max, off);
  o.minidx = __shfl_down(r.minidx, off);
  o.maxidx = __shfl_down(r.maxidx, off);
  o.count = __shfl_down(r.count, off);
  o.ymin = __shfl_down(r.ymin, off);
  return o;
}

// The kernel of Eq. 4 between a training point (global memory) and the
// chosen point (LDS), each M points of D coordinates (D = 3: control points and
// K_FK; M = 1, D = n: the joint vector and the kernel of Eq. 3 on
// configurations), with direct differences. The FP64 form disables FMA
// contraction so that it rounds operation by operation in the order the
// definition is written.
__device__ __forceinline__ float kfk_pair(const float* __restrict__ pj, const float* pi, int M, int D, float half_g) {
  float s = 0.f;
  if (D == 3) {
    for (int m = 0; m < M; ++m) {
      const float dx = pj[3 * m] - pi[3 * m], dy = pj[3 * m + 1] - pi[3 * m + 1], dz = pj[3 * m + 2] - pi[3 * m + 2];
      const float t = 1.0f + half_g * (dx * dx + dy * dy + dz * dz);
      const float r = __builtin_amdgcn_rcpf(t);
      s = fmaf(r, r, s);
    }
  } else {
    for (int m = 0; m < M; ++m) {
      float d2 = 0.f;
      for (int k = 0; k < D; ++k) {
        const float diff = pj[D * m + k] - pi[D * m + k];
        d2 = fmaf(diff, diff, d2);
      }
      const float r = __builtin_amdgcn_rcpf(1.0f + half_g * d2);
      s = fmaf(r, r, s);
    }
  }
  return s / (float)M;
}

__device__ __forceinline__ double kfk_pair(const float* __restrict__ pj, const float* pi, int M, int D,
                                           double half_g) {
#pragma clang fp contract(off)
  double s = 0.0;
  for (int m = 0; m < M; ++m) {
    double d2 = 0.0;
    for (int k = 0; k < D; ++k) {
      const double diff = (double)pj[D * m + k] - (double)pi[D * m + k];
      d2 += diff * diff;
    }
    const double t = 1.0 + half_g * d2;
    s += 1.0 / (t * t);
  }
  return s / (double)M;
}

// The same K_FK with both points' coordinates in registers (MM points,
// compile-time), evaluated in the same order as kfk_pair.
template <int MM>
__device__ __forceinline__ float kfk_regs(const float* pj, const float* pi, float half_g) {
  float s = 0.f;
#pragma unroll
  for (int m = 0; m < MM; ++m) {
    const float dx = pj[3 * m] - pi[3 * m], dy = pj[3 * m + 1] - pi[3 * m + 1], dz = pj[3 * m + 2] - pi[3 * m + 2];
    const float t = 1.0f + half_g * (dx * dx + dy * dy + dz * dz);
    const float r = __builtin_amdgcn_rcpf(t);
    s = fmaf(r, r, s);
  }
  return s / (float)MM;
}

template <int MM>
__device__ __forceinline__ double kfk_regs(const float* pj, const float* pi, double half_g) {
#pragma clang fp contract(off)
  double s = 0.0;
#pragma unroll
  for (int m = 0; m < MM; ++m) {
    double d2 = 0.0;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const double diff = (double)pj[3 * m + k] - (double)pi[3 * m + k];
      d2 += diff * diff;
    }
    const double t = 1.0 + half_g * d2;
    s += 1.0 / (t * t);
  }
  return s / (double)MM;
}

__device__ __forceinline__ float axpy_rn(float a, float x, float y) { return y + a * x; }

// ---------------------------------------------------------------------------
// a4: Gram column + F update, one thread per training point.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_gram_update(const float* __restrict__ P, int64_t N, int M, float half_g,
                                                      int64_t i, float dalpha, float* __restrict__ F,
                                                      float* __restrict__ kcol) {
  __shared__ float pi_sh[3 * FASTRON_MAX_POINTS];
  if ((int)threadIdx.x < 3 * M) pi_sh[threadIdx.x] = P[i * (int64_t)M * 3 + threadIdx.x];
  __syncthreads();
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (j >= N) return;
  const float k = kfk_pair(P + j * (int64_t)M * 3, pi_sh, M, 3, half_g);
  if (kcol) kcol[j] = k;
  if (F) F[j] = axpy_rn(dalpha, k, F[j]);
}
__device__ __forceinline__ double axpy_rn(double a, double x, double y) {
#pragma clang fp contract(off)
  return y + a * x;
}
__device__ __forceinline__ float sub_rn(float a, float b) { return a - b; }
__device__ __forceinline__ double sub_rn(double a, double b) {
#pragma clang fp contract(off)
  return a - b;
}

// Decision shared by the workgroup after each reduction.
template <typename T>
struct Decision {
  T dalpha;
  int64_t i;
  int action;  // 1 add, 2 remove, 0 break (converged), 3 stop (iter_max), 4 stop (exchange timeout)
};

template <typename T>
__device__ __forceinline__ Rec<T> wave_reduce(Rec<T> r) {
  for (int off = 32; off > 0; off >>= 1) {
    Rec<T> o = rec_shfl_down(r, off);
    if ((int)(threadIdx.x & 63) + off < 64) rec_merge(r, o);
  }
  return r;
}

template <typename T>
__device__ __forceinline__ void point_record(Rec<T>& r, int64_t j, T yj, T Fj, T aj) {
  Rec<T> c = rec_empty<T>();
  c.minval = yj * Fj;
  c.a_at_min = aj;
  c.minidx = (int32_t)j;
  c.ymin = yj > (T)0 ? 1 : -1;
  if (aj != (T)0) {
    c.maxval = yj * (Fj - aj);
    c.a_at_max = aj;
    c.maxidx = (int32_t)j;
    c.count = 1;
  }
  rec_merge(r, c);
}

// Record exchange without a central barrier: a record is published as K
// 64-bit words, each holding 56 payload bits under an 8-bit tag, the low
// byte of the iteration number + 1. A word is stored and loaded with
// single-copy-atomic, device-coherent 64-bit accesses, so a reader that sees
// the current tag in every word of a record has the whole record; no fence or
// read-modify-write is needed. Records are double-buffered by iteration
// parity: a workgroup cannot publish iteration it + 2 before every workgroup
// has published iteration it + 1, which each does only after reading
// iteration it. The slot a reader polls at iteration it therefore holds the
// writer's word of iteration it - 2 (which this reader has already read, so
// nothing older can come back) or of iteration it, or for it < 2 the zeros
// written before the launch; their tags differ modulo 256.
__device__ __forceinline__ unsigned long long rec_tag(int64_t it) {
  return (unsigned long long)((it + 1) & 0xff) << 56;
}
__device__ __forceinline__ bool rec_tagged(unsigned long long w, unsigned long long tag) {
  return (w & 0xff00000000000000ull) == tag;
}

template <typename T>
struct RecWords;
// FP32 record in 4 words: each word carries one of the four values (32 bits)
// and the low 24 bits of one of the three 31-bit integers minidx + 1,
// maxidx + 1 and count (indices and counts are below 2^31 - 1); word 3 carries
// their top 7 bits and the label bit instead.
template <>
struct RecWords<float> {
  static constexpr int K = 4;
  __device__ static unsigned long long get(const Rec<float>& r, int k) {
    const unsigned long long mi = (uint32_t)(r.minidx + 1), xi = (uint32_t)(r.maxidx + 1), c = (uint32_t)r.count;
    switch (k) {
      case 0: return __float_as_uint(r.minval) | ((mi & 0xffffff) << 32);
      case 1: return __float_as_uint(r.a_at_min) | ((xi & 0xffffff) << 32);
      case 2: return __float_as_uint(r.maxval) | ((c & 0xffffff) << 32);
      default:
        return __float_as_uint(r.a_at_max) |
               (((mi >> 24) | ((xi >> 24) << 7) | ((c >> 24) << 14) | ((r.ymin > 0 ? 1ull : 0ull) << 21)) << 32);
    }
  }
  __device__ static Rec<float> make(const unsigned long long* w) {
    const uint32_t h = (uint32_t)(w[3] >> 32) & 0xffffff;
    Rec<float> r;
    r.minval = __uint_as_float((uint32_t)w[0]);
    r.a_at_min = __uint_as_float((uint32_t)w[1]);
    r.maxval = __uint_as_float((uint32_t)w[2]);
    r.a_at_max = __uint_as_float((uint32_t)w[3]);
    r.minidx = (int32_t)((((uint32_t)(w[0] >> 32)) & 0xffffff) | ((h & 0x7f) << 24)) - 1;
    r.maxidx = (int32_t)((((uint32_t)(w[1] >> 32)) & 0xffffff) | (((h >> 7) & 0x7f) << 24)) - 1;
    r.count = (int32_t)((((uint32_t)(w[2] >> 32)) & 0xffffff) | (((h >> 14) & 0x7f) << 24));
    r.ymin = ((h >> 21) & 1) ? 1 : -1;
    return r;
  }
};
// FP64 record in 7 words: words 0-3 the low 56 bits of the four values, word 4
// their top bytes and 24 bits of minidx + 1, word 5 maxidx + 1 and 25 bits of
// the count, word 6 the remaining bits and the label bit.
template <>
struct RecWords<double> {
  static constexpr int K = 7;
  static constexpr unsigned long long kLow56 = (1ull << 56) - 1;
  __device__ static unsigned long long bits(double v) { return (unsigned long long)__double_as_longlong(v); }
  __device__ static unsigned long long get(const Rec<double>& r, int k) {
    const unsigned long long mi = (uint32_t)(r.minidx + 1), xi = (uint32_t)(r.maxidx + 1), c = (uint32_t)r.count;
    switch (k) {
      case 0: return bits(r.minval) & kLow56;
      case 1: return bits(r.a_at_min) & kLow56;
      case 2: return bits(r.maxval) & kLow56;
      case 3: return bits(r.a_at_max) & kLow56;
      case 4:
        return (bits(r.minval) >> 56) | ((bits(r.a_at_min) >> 56) << 8) | ((bits(r.maxval) >> 56) << 16) |
               ((bits(r.a_at_max) >> 56) << 24) | ((mi & 0xffffff) << 32);
      case 5: return xi | ((c & 0x1ffffff) << 31);
      default: return (mi >> 24) | ((c >> 25) << 7) | ((r.ymin > 0 ? 1ull : 0ull) << 13);
    }
  }
  __device__ static double join(unsigned long long lo, unsigned long long top) {
    return __longlong_as_double((long long)((lo & kLow56) | ((top & 0xff) << 56)));
  }
  __device__ static Rec<double> make(const unsigned long long* w) {
    Rec<double> r;
    r.minval = join(w[0], w[4]);
    r.a_at_min = join(w[1], w[4] >> 8);
    r.maxval = join(w[2], w[4] >> 16);
    r.a_at_max = join(w[3], w[4] >> 24);
    r.minidx = (int32_t)(((uint32_t)(w[4] >> 32) & 0xffffff) | (((uint32_t)w[6] & 0x7f) << 24)) - 1;
    r.maxidx = (int32_t)((uint32_t)w[5] & 0x7fffffff) - 1;
    r.count = (int32_t)(((uint32_t)(w[5] >> 31) & 0x1ffffff) | ((((uint32_t)w[6] >> 7) & 0x3f) << 25));
    r.ymin = (((uint32_t)w[6] >> 13) & 1) ? 1 : -1;
    return r;
  }
};

// One workgroup per slice; PT training points per thread, their y, alpha and
// F held in registers for the whole run. Wave 0 leads: it publishes the
// workgroup's record, gathers every workgroup's record of the same iteration,
// reduces them and broadcasts the decision (and the chosen point's control
// points) through LDS. Every workgroup reduces the same records in the same
// way, so all take the same decision.
template <typename T, int PT>
__global__ void __launch_bounds__(1024) k_train(TrainState<T> st) {
  constexpr int K = RecWords<T>::K;
  __shared__ Rec<T> sh[16];
  __shared__ Decision<T> dec;
  __shared__ float pi_sh[3 * FASTRON_MAX_POINTS];
  extern __shared__ float pslice[];  // this slice's control points when they fit (st.p_in_lds)
  const unsigned G = gridDim.x;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const int64_t j0 = (int64_t)blockIdx.x * st.chunk;
  const int64_t j1 = (j0 + st.chunk < st.N) ? j0 + st.chunk : st.N;
  const int M = st.M, W = M * st.D;  // floats per training point
  if (st.p_in_lds)
    for (int64_t e = threadIdx.x; e < (j1 - j0) * W; e += blockDim.x) pslice[e] = st.P[j0 * W + e];
  unsigned long long* words = reinterpret_cast<unsigned long long*>(st.rec);  // [2][G][K]

  T y[PT], F[PT], a[PT];
  int64_t jj[PT];
  Rec<T> r = rec_empty<T>();
#pragma unroll
  for (int k = 0; k < PT; ++k) {
    jj[k] = j0 + threadIdx.x + (int64_t)k * blockDim.x;
    if (jj[k] < j1) {
      y[k] = (T)st.y[jj[k]];
      F[k] = st.F[jj[k]];
      a[k] = st.alpha[jj[k]];
      point_record(r, jj[k], y[k], F[k], a[k]);
    } else {
      y[k] = 0;
      F[k] = 0;
      a[k] = 0;
    }
  }
  r = wave_reduce(r);
  if (lane == 0) sh[wave] = r;
  __syncthreads();

  int64_t updates = 0;
  int64_t status = 1;
  for (int64_t it = 0;; ++it) {
    if (wave == 0) {
      Rec<T> mine = sh[0];
      for (int w = 1; w < nw; ++w) rec_merge(mine, sh[w]);
      const unsigned long long tag = rec_tag(it);
      unsigned long long* slot = words + (size_t)(it & 1) * G * K;
      if (lane < K)
        __hip_atomic_store(slot + (size_t)blockIdx.x * K + lane, tag | RecWords<T>::get(mine, lane),
                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      // gather: lane l reads records l, l + 64, ...
      Rec<T> gr = rec_empty<T>();
      bool ok = true;
      for (unsigned base = 0; base < G; base += 64) {
        const unsigned w = base + lane;
        unsigned long long pay[K];
        bool ready = w >= G;
        const long long t0 = wall_clock64();
        while (true) {
          if (!ready) {
            ready = true;
#pragma unroll
            for (int k = 0; k < K; ++k) {
              const unsigned long long v =
                  __hip_atomic_load(slot + (size_t)w * K + k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
              pay[k] = v;
              ready = ready && rec_tagged(v, tag);
            }
          }
          if (__all(ready)) break;
          __builtin_amdgcn_s_sleep(1);
          if (wall_clock64() - t0 > st.timeout) {
            ok = false;
            break;
          }
        }
        if (!__all(ok)) {
          ok = false;
          break;
        }
        if (w < G) rec_merge(gr, RecWords<T>::make(pay));
      }
      gr = wave_reduce(gr);
      gr.minval = __shfl(gr.minval, 0);
      gr.a_at_min = __shfl(gr.a_at_min, 0);
      gr.maxval = __shfl(gr.maxval, 0);
      gr.a_at_max = __shfl(gr.a_at_max, 0);
      gr.minidx = __shfl(gr.minidx, 0);
      gr.maxidx = __shfl(gr.maxidx, 0);
      gr.count = __shfl(gr.count, 0);
      gr.ymin = __shfl(gr.ymin, 0);
      Decision<T> d;
      d.action = 0;
      d.i = -1;
      d.dalpha = 0;
      if (!ok) {
        d.action = 4;
      } else if (updates >= st.iter_max) {
        d.action = 3;
      } else if (gr.minidx >= 0 && gr.minval <= (T)0 && ((int64_t)gr.count < st.s_max || gr.a_at_min != (T)0)) {
        d.i = gr.minidx;
        const T yi = (T)gr.ymin;
        const T Fi = yi * gr.minval;          // y = +-1: y (y F) = F exactly
        const T bi = yi > 0 ? st.beta : (T)1;  // b_i = beta^(0.5 (y_i + 1)), Eq. 5
        d.dalpha = sub_rn(bi * yi, Fi);        // Eq. 6
        d.action = 1;
      } else if (gr.maxidx >= 0 && gr.maxval > (T)0) {
        d.i = gr.maxidx;
        d.dalpha = -gr.a_at_max;
        d.action = 2;
      }
      if (d.action == 1 || d.action == 2) {
        if (lane < W) pi_sh[lane] = st.P[d.i * (int64_t)W + lane];
        if (blockIdx.x == 0 && lane == 0 && updates < st.trace_cap) {
          st.trace_act[updates] = d.action;
          st.trace_idx[updates] = (int32_t)d.i;
        }
      }
      if (lane == 0) dec = d;
    }
    __syncthreads();
    const Decision<T> d = dec;
    if (d.action != 1 && d.action != 2) {
      status = d.action == 0 ? 0 : (d.action == 3 ? 1 : -5);
      break;
    }
    ++updates;
    // column i of K on this thread's points (Eq. 8), fused with the next record
    r = rec_empty<T>();
#pragma unroll
    for (int k = 0; k < PT; ++k) {
      if (jj[k] < j1) {
        // index the LDS slice relative to its own start (pointer arithmetic stays inside each object)
        const float* pj = st.p_in_lds ? pslice + (jj[k] - j0) * (int64_t)W : st.P + jj[k] * (int64_t)W;
        const T kv = kfk_pair(pj, pi_sh, M, st.D, st.half_g);
        F[k] = axpy_rn(d.dalpha, kv, F[k]);
        if (jj[k] == d.i) a[k] = (d.action == 1) ? a[k] + d.dalpha : (T)0;  // Eq. 7 / removal
        point_record(r, jj[k], y[k], F[k], a[k]);
      }
    }
    r = wave_reduce(r);
    if (lane == 0) sh[wave] = r;
    __syncthreads();
  }
#pragma unroll
  for (int k = 0; k < PT; ++k)
    if (jj[k] < j1) {
      st.F[jj[k]] = F[k];
      st.alpha[jj[k]] = a[k];
    }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    st.out[0] = updates;
    st.out[1] = status;
  }
}

// Whole-wave reduction of records (or of the first row of 16 lanes, the
// first four steps only); every lane ends with the result. The
// (value, index) pairs are compared lexicographically (lowest index on ties)
// and the counts summed along the DPP sequence quad_perm [1,0,3,2],
// quad_perm [2,3,0,1], row_half_mirror, row_mirror (after which every lane of
// a row of 16 holds its row's result), row_bcast:15 into rows 1 and 3 and
// row_bcast:31 into rows 2 and 3, so that lane 63 holds the wave's result
// (lane 0 the row's); no step goes through LDS. The fields are read from that
// lane and the payloads
// (weights, label) from the lane whose own record holds the winning index
// (indices are unique across the lanes' records).
template <int CTRL, int ROWS>
__device__ __forceinline__ int dpp_keep(int v) {  // lanes outside ROWS keep their own value
  if constexpr (ROWS == 0xf)
    return __builtin_amdgcn_mov_dpp(v, CTRL, 0xf, 0xf, true);  // every lane written: no copy of v first
  else
    return __builtin_amdgcn_update_dpp(v, v, CTRL, ROWS, 0xf, false);
}
template <int CTRL, int ROWS>
__device__ __forceinline__ int dpp_zero(int v) {  // lanes outside ROWS read 0
  return __builtin_amdgcn_update_dpp(0, v, CTRL, ROWS, 0xf, false);
}
template <int CTRL, int ROWS>
__device__ __forceinline__ unsigned long long dpp_keep64(unsigned long long v) {
  const uint32_t lo = (uint32_t)dpp_keep<CTRL, ROWS>((int)(uint32_t)v);
  const uint32_t hi = (uint32_t)dpp_keep<CTRL, ROWS>((int)(uint32_t)(v >> 32));
  return ((unsigned long long)hi << 32) | lo;
}
__device__ __forceinline__ unsigned long long readlane64(unsigned long long v, int l) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, l);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), l);
  return ((unsigned long long)hi << 32) | lo;
}
__device__ __forceinline__ float readlane(float v, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}
__device__ __forceinline__ double readlane(double v, int l) {
  return __longlong_as_double((long long)readlane64((unsigned long long)__double_as_longlong(v), l));
}

// FP32 records, in two passes of single DPP-modified min / max / add
// instructions. Pass 1 reduces the values, mapped to an unsigned
// order-preserving form (-0 taken as +0 since the two compare equal; an empty
// half maps to the form that never wins), and the counts; pass 2 reduces the
// indices of the lanes whose value equals the winner (the lowest index wins a
// tie, for the min and the max alike).
__device__ __forceinline__ uint32_t ordered_bits(float v) {
  const uint32_t u = v == 0.f ? 0u : __float_as_uint(v);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
// Lanes outside ROWS read the operation's identity, so each step is one
// DPP-modified instruction.
template <int CTRL, int ROWS>
__device__ __forceinline__ uint32_t dpp_ident(uint32_t v, uint32_t ident) {
  if constexpr (ROWS == 0xf)
    return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, CTRL, 0xf, 0xf, true);
  else
    return (uint32_t)__builtin_amdgcn_update_dpp((int)ident, (int)v, CTRL, ROWS, 0xf, false);
}
template <int CTRL, int ROWS>
__device__ __forceinline__ void value_step(uint32_t& vmin, uint32_t& vmax, int& cnt) {
  const uint32_t omin = dpp_ident<CTRL, ROWS>(vmin, 0xffffffffu), omax = dpp_ident<CTRL, ROWS>(vmax, 0u);
  cnt += dpp_zero<CTRL, ROWS>(cnt);
  vmin = omin < vmin ? omin : vmin;
  vmax = omax > vmax ? omax : vmax;
}
template <int CTRL, int ROWS>
__device__ __forceinline__ void index_step(uint32_t& imin, uint32_t& imax) {
  const uint32_t omin = dpp_ident<CTRL, ROWS>(imin, 0xffffffffu), omax = dpp_ident<CTRL, ROWS>(imax, 0xffffffffu);
  imin = omin < imin ? omin : imin;
  imax = omax < imax ? omax : imax;
}
// The two passes; every lane ends with the winners' ordered values and
// indices (kNoIndex for an empty half) and the count.
constexpr uint32_t kNoIndex = 0x7fffffffu;
template <int LANES>
__device__ __forceinline__ void wave_winners(const Rec<float>& r, uint32_t& vmin, uint32_t& imin, uint32_t& vmax,
                                             uint32_t& imax, int& cnt) {
  static_assert(LANES == 64 || LANES == 16, "whole wave or its first row");
  constexpr int kOut = LANES == 64 ? 63 : 0;  // the lane that ends with the result
  const uint32_t mine_min = r.minidx < 0 ? 0xffffffffu : ordered_bits(r.minval);
  const uint32_t mine_max = r.maxidx < 0 ? 0u : ordered_bits(r.maxval);
  vmin = mine_min;
  vmax = mine_max;
  cnt = r.count;
  value_step<0xB1, 0xf>(vmin, vmax, cnt);
  value_step<0x4E, 0xf>(vmin, vmax, cnt);
  value_step<0x141, 0xf>(vmin, vmax, cnt);
  value_step<0x140, 0xf>(vmin, vmax, cnt);
  if constexpr (LANES == 64) {
    value_step<0x142, 0xa>(vmin, vmax, cnt);
    value_step<0x143, 0xc>(vmin, vmax, cnt);
  }
  vmin = (uint32_t)__builtin_amdgcn_readlane((int)vmin, kOut);
  vmax = (uint32_t)__builtin_amdgcn_readlane((int)vmax, kOut);
  imin = (r.minidx >= 0 && mine_min == vmin) ? (uint32_t)r.minidx : kNoIndex;
  imax = (r.maxidx >= 0 && mine_max == vmax) ? (uint32_t)r.maxidx : kNoIndex;
  index_step<0xB1, 0xf>(imin, imax);
  index_step<0x4E, 0xf>(imin, imax);
  index_step<0x141, 0xf>(imin, imax);
  index_step<0x140, 0xf>(imin, imax);
  if constexpr (LANES == 64) {
    index_step<0x142, 0xa>(imin, imax);
    index_step<0x143, 0xc>(imin, imax);
  }
  imin = (uint32_t)__builtin_amdgcn_readlane((int)imin, kOut);
  imax = (uint32_t)__builtin_amdgcn_readlane((int)imax, kOut);
  cnt = __builtin_amdgcn_readlane(cnt, kOut);
}
template <int LANES = 64>
__device__ __forceinline__ Rec<float> wave_allreduce(const Rec<float>& r) {
  uint32_t vmin, imin, vmax, imax;
  int cnt;
  wave_winners<LANES>(r, vmin, imin, vmax, imax, cnt);
  Rec<float> o = rec_empty<float>();
  o.count = cnt;
  if (imin != kNoIndex) {
    const int mi = (int)imin;
    const int src = __builtin_ctzll(__ballot(r.minidx == mi));
    o.minidx = mi;
    o.minval = readlane(r.minval, src);
    o.a_at_min = readlane(r.a_at_min, src);
    o.ymin = __builtin_amdgcn_readlane(r.ymin, src);
  }
  if (imax != kNoIndex) {
    const int xi = (int)imax;
    const int src = __builtin_ctzll(__ballot(r.maxidx == xi));
    o.maxidx = xi;
    o.maxval = readlane(r.maxval, src);
    o.a_at_max = readlane(r.a_at_max, src);
  }
  return o;
}

// Workgroup keys of FP32 records: the wave's winners as two unsigned 64-bit
// keys whose order is the records' order (ordered value above, index below
// for the min, 2^31 - 1 - index below for the max; the empty key never wins),
// combined across waves with LDS atomic min / max.
__device__ __forceinline__ unsigned long long min_key(uint32_t v, uint32_t i) {
  return i == kNoIndex ? ~0ull : ((unsigned long long)v << 32) | i;
}
__device__ __forceinline__ unsigned long long max_key(uint32_t v, uint32_t i) {
  return i == kNoIndex ? 0ull : ((unsigned long long)v << 32) | (kNoIndex - i);
}
__device__ __forceinline__ float from_ordered(uint32_t o) {
  return __uint_as_float((o & 0x80000000u) ? (o & 0x7fffffffu) : ~o);
}

// FP64 records: the values compared as doubles (DPP moves of both halves).
template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_keep(double v) {
  return __longlong_as_double((long long)dpp_keep64<CTRL, ROWS>((unsigned long long)__double_as_longlong(v)));
}
template <int CTRL, int ROWS>
__device__ __forceinline__ void pair_step(double& mv, int& mi, double& xv, int& xi, int& cnt) {
  const double omv = dpp_keep<CTRL, ROWS>(mv), oxv = dpp_keep<CTRL, ROWS>(xv);
  const int omi = dpp_keep<CTRL, ROWS>(mi), oxi = dpp_keep<CTRL, ROWS>(xi);
  cnt += dpp_zero<CTRL, ROWS>(cnt);
  const bool tmin = omi >= 0 && (mi < 0 || omv < mv || (omv == mv && omi < mi));
  const bool tmax = oxi >= 0 && (xi < 0 || oxv > xv || (oxv == xv && oxi < xi));
  mv = tmin ? omv : mv;
  mi = tmin ? omi : mi;
  xv = tmax ? oxv : xv;
  xi = tmax ? oxi : xi;
}
template <int LANES = 64>
__device__ __forceinline__ Rec<double> wave_allreduce(const Rec<double>& r) {
  static_assert(LANES == 64 || LANES == 16, "whole wave or its first row");
  constexpr int kOut = LANES == 64 ? 63 : 0;
  double mv = r.minval, xv = r.maxval;
  int mi = r.minidx, xi = r.maxidx, cnt = r.count;
  pair_step<0xB1, 0xf>(mv, mi, xv, xi, cnt);
  pair_step<0x4E, 0xf>(mv, mi, xv, xi, cnt);
  pair_step<0x141, 0xf>(mv, mi, xv, xi, cnt);
  pair_step<0x140, 0xf>(mv, mi, xv, xi, cnt);
  if constexpr (LANES == 64) {
    pair_step<0x142, 0xa>(mv, mi, xv, xi, cnt);
    pair_step<0x143, 0xc>(mv, mi, xv, xi, cnt);
  }
  mi = __builtin_amdgcn_readlane(mi, kOut);
  xi = __builtin_amdgcn_readlane(xi, kOut);
  Rec<double> o = rec_empty<double>();
  o.count = __builtin_amdgcn_readlane(cnt, kOut);
  if (mi >= 0) {
    const int src = __builtin_ctzll(__ballot(r.minidx == mi));
    o.minidx = mi;
    o.minval = readlane(r.minval, src);
    o.a_at_min = readlane(r.a_at_min, src);
    o.ymin = __builtin_amdgcn_readlane(r.ymin, src);
  }
  if (xi >= 0) {
    const int src = __builtin_ctzll(__ballot(r.maxidx == xi));
    o.maxidx = xi;
    o.maxval = readlane(r.maxval, src);
    o.a_at_max = readlane(r.a_at_max, src);
  }
  return o;
}

// Wave form of the same algorithm. No workgroup barrier stands inside the
// record exchange: one wave (wave 0) publishes the workgroup's record and
// gathers the others, each lane reading the records of workgroups lane,
// lane + 64, ... (issuing the loads of all its records before checking their
// tags), and records are reduced with DPP row operations. MULTI = false: single-wave
// workgroups (up to kWaveChunks x 64 of them). MULTI = true: workgroups of
// blockDim.x / 64 waves (up to 16 / PT, so that a grid of a few dozen
// workgroups covers a large training set: the exchange's cost grows with the
// number of records every workgroup reads); the waves' records meet in LDS,
// wave 0 exchanges their merge and broadcasts the decision, so an iteration
// takes two workgroup barriers (up to kMultiChunks x 64 workgroups).
constexpr int kWaveChunks = 8;
constexpr int kMaxPollDelay = 64;  // sleeps before the first poll (about 2 us)
template <typename T>
constexpr int kMultiChunks = sizeof(T) == 4 ? 4 : 2;  // FP64 records take twice the registers
constexpr int kMultiMaxPT = 4;  // points per lane of multi-wave workgroups in multi-set launches (FP32)

// MM > 0: the chain has exactly MM control points and every lane keeps its
// points' coordinates in registers for the whole run; MM = 0: any M, the
// coordinates come from LDS (or global memory) in each column pass.
template <typename T, int PT, int MM, bool MULTI>
__global__ void __launch_bounds__(MULTI ? (sizeof(T) == 8 ? 512 : 1024 / PT) : 64) k_train_wave(TrainState<T> st) {
  constexpr int K = RecWords<T>::K;
  constexpr int CH = MULTI ? kMultiChunks<T> : kWaveChunks;
  // FP32 with several waves: the waves' records meet as LDS keys and per-lane
  // payloads (see min_key); FP64: as whole records reduced by wave 0.
  constexpr bool kKeys = MULTI && sizeof(T) == 4;
  constexpr int kLanes = kKeys ? 1024 / PT : 1;
  __shared__ float pi_sh[3 * FASTRON_MAX_POINTS];
  __shared__ Rec<T> sh[MULTI ? 16 : 1];
  __shared__ Decision<T> dec;
  __shared__ unsigned long long sh_kmin, sh_kmax;
  __shared__ int sh_cnt;
  __shared__ T sh_amin[kLanes], sh_amax[kLanes];
  __shared__ int8_t sh_ymin[kLanes];
  extern __shared__ float pslice[];  // this slice's control points when they fit (st.p_in_lds)
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int nt = MULTI ? (int)blockDim.x : 64, nw = nt >> 6;
  // this workgroup's training set: its workgroups (G, own index me), points and records
  unsigned G = gridDim.x, me = blockIdx.x;
  int64_t set_lo = 0, set_hi = st.N;
  unsigned long long* words = reinterpret_cast<unsigned long long*>(st.rec);  // [2][G][K] per set
  int64_t* out = st.out;
  if (st.env_of) {
    const int e = st.env_of[blockIdx.x];
    const int w0 = st.env_wg0[e];
    G = (unsigned)(st.env_wg0[e + 1] - w0);
    me = blockIdx.x - (unsigned)w0;
    set_lo = st.env_off[e];
    set_hi = st.env_off[e + 1];
    words += (size_t)2 * K * w0;
    out += 2 * e;
  }
  const int64_t j0 = set_lo + (int64_t)me * st.chunk;  // chunk = nt * PT
  const int64_t j1 = (j0 + st.chunk < set_hi) ? j0 + st.chunk : set_hi;
  const int M = st.M, W = M * st.D;  // floats per training point
  if (st.p_in_lds)
    for (int64_t e = threadIdx.x; e < (j1 - j0) * W; e += nt) pslice[e] = st.P[j0 * W + e];
  if (threadIdx.x == 0) {
    sh_kmin = ~0ull;
    sh_kmax = 0ull;
    sh_cnt = 0;
  }
  __syncthreads();

  T y[PT], F[PT], a[PT];
  int64_t jj[PT];
  constexpr int kReg = MM > 0 ? 3 * MM : 1;
  float pjr[PT][kReg];
  Rec<T> r = rec_empty<T>();
#pragma unroll
  for (int k = 0; k < PT; ++k) {
    jj[k] = j0 + threadIdx.x + (int64_t)k * nt;
#pragma unroll
    for (int e = 0; e < kReg; ++e) pjr[k][e] = 0.f;
    if (jj[k] < j1) {
      y[k] = (T)st.y[jj[k]];
      F[k] = st.F[jj[k]];
      a[k] = st.alpha[jj[k]];
      if constexpr (MM > 0) {
#pragma unroll
        for (int e = 0; e < kReg; ++e) pjr[k][e] = st.P[jj[k] * kReg + e];
      }
      point_record(r, jj[k], y[k], F[k], a[k]);
    } else {
      y[k] = 0;
      F[k] = 0;
      a[k] = 0;
    }
  }
  if constexpr (!kKeys) r = wave_allreduce(r);

  int64_t updates = 0;
  int64_t status = 1;
  // Sleeps before the first poll of an exchange. A poll that finds a record
  // missing costs a whole memory round trip, and right after publishing the
  // other workgroups' records are rarely all visible yet, so the first poll
  // waits. Adaptive (poll_delay < 0): two more sleeps after an exchange whose
  // first poll came too early, one fewer after four in a row that did not,
  // which settles where about nine first polls in ten find every record.
  int delay = st.poll_delay < 0 ? 8 : st.poll_delay, early_ok = 0;
  for (int64_t it = 0;; ++it) {
    if constexpr (kKeys) {
      // r is this lane's record: payload to LDS, the wave's keys into the workgroup's
      if constexpr (sizeof(T) == 4) {
        sh_amin[threadIdx.x] = r.a_at_min;
        sh_amax[threadIdx.x] = r.a_at_max;
        sh_ymin[threadIdx.x] = (int8_t)r.ymin;
        uint32_t vmin, imin, vmax, imax;
        int cnt;
        wave_winners<64>(r, vmin, imin, vmax, imax, cnt);
        if (lane == 0) {
          atomicMin(&sh_kmin, min_key(vmin, imin));
          atomicMax(&sh_kmax, max_key(vmax, imax));
          atomicAdd(&sh_cnt, cnt);
        }
      }
      __syncthreads();  // the workgroup's keys are complete; every wave is done with pi_sh and dec
    } else if constexpr (MULTI) {
      if (lane == 0) sh[wave] = r;
      __syncthreads();  // the waves' records are in LDS; every wave is done with pi_sh and dec
    }
    Decision<T> d;
    if (!MULTI || wave == 0) {
      Rec<T> mine = r;
      if constexpr (kKeys) {
        // the winners' payloads sit at their lanes: index j is held by thread (j - j0) mod nt
        const unsigned long long kmin = sh_kmin, kmax = sh_kmax;
        mine = rec_empty<T>();
        mine.count = sh_cnt;
        if (kmin != ~0ull) {
          const int mi = (int)(uint32_t)kmin;
          const int pos = (int)((mi - j0) & (nt - 1));
          mine.minidx = mi;
          mine.minval = from_ordered((uint32_t)(kmin >> 32));
          mine.a_at_min = sh_amin[pos];
          mine.ymin = sh_ymin[pos];
        }
        if (kmax != 0ull) {
          const int xi = (int)(kNoIndex - (uint32_t)kmax);
          const int pos = (int)((xi - j0) & (nt - 1));
          mine.maxidx = xi;
          mine.maxval = from_ordered((uint32_t)(kmax >> 32));
          mine.a_at_max = sh_amax[pos];
        }
        if (lane == 0) {  // after this wave's reads; the next atomics follow the second barrier
          sh_kmin = ~0ull;
          sh_kmax = 0ull;
          sh_cnt = 0;
        }
      } else if constexpr (MULTI) {
        mine = wave_allreduce<16>(lane < nw ? sh[lane] : rec_empty<T>());
      }
      Rec<T> gr = rec_empty<T>();
      bool ok = true;
      if (G == 1) {
        gr = mine;  // the set's only workgroup: its record is the set's, nothing to exchange
      } else {
        const unsigned long long tag = rec_tag(it);
        unsigned long long* slot = words + (size_t)(it & 1) * G * K;
        if (lane < K)
          __hip_atomic_store(slot + (size_t)me * K + lane, tag | RecWords<T>::get(mine, lane), __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_AGENT);
        unsigned long long pay[CH][K];
        bool ready[CH];
#pragma unroll
        for (int c = 0; c < CH; ++c) ready[c] = c * 64 + lane >= (int)G;
        for (int q = 0; q < delay; ++q) __builtin_amdgcn_s_sleep(1);
        int polls = 0;
        const long long t0 = wall_clock64();
        while (true) {
          ++polls;
          bool all = true;
#pragma unroll
          for (int c = 0; c < CH; ++c) {
            if (!ready[c]) {
              const unsigned long long* rw = slot + (size_t)(c * 64 + lane) * K;
              bool rd = true;
#pragma unroll
              for (int k = 0; k < K; ++k) {
                pay[c][k] = __hip_atomic_load(rw + k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                rd = rd && rec_tagged(pay[c][k], tag);
              }
              ready[c] = rd;
            }
            all = all && ready[c];
          }
          if (__all(all)) break;
          __builtin_amdgcn_s_sleep(1);
          if (wall_clock64() - t0 > st.timeout) {
            ok = false;
            break;
          }
        }
        if (st.poll_delay < 0) {
          if (polls > 1) {
            delay = delay + 2 < kMaxPollDelay ? delay + 2 : kMaxPollDelay;
            early_ok = 0;
          } else if (++early_ok == 4) {
            delay = delay > 0 ? delay - 1 : 0;
            early_ok = 0;
          }
        }
        if (ok) {
#pragma unroll
          for (int c = 0; c < CH; ++c)
            if (c * 64 < (int)G && c * 64 + lane < (int)G) rec_merge(gr, RecWords<T>::make(pay[c]));
          gr = wave_allreduce(gr);
        }
      }
      d.action = 0;
      d.i = -1;
      d.dalpha = 0;
      if (!ok) {
        d.action = 4;
      } else if (updates >= st.iter_max) {
        d.action = 3;
      } else if (gr.minidx >= 0 && gr.minval <= (T)0 && ((int64_t)gr.count < st.s_max || gr.a_at_min != (T)0)) {
        d.i = gr.minidx;
        const T yi = (T)gr.ymin;
        const T Fi = yi * gr.minval;          // y = +-1: y (y F) = F exactly
        const T bi = yi > 0 ? st.beta : (T)1;  // b_i = beta^(0.5 (y_i + 1)), Eq. 5
        d.dalpha = sub_rn(bi * yi, Fi);        // Eq. 6
        d.action = 1;
      } else if (gr.maxidx >= 0 && gr.maxval > (T)0) {
        d.i = gr.maxidx;
        d.dalpha = -gr.a_at_max;
        d.action = 2;
      }
      if (d.action == 1 || d.action == 2) {
        if (lane < W) pi_sh[lane] = st.P[d.i * (int64_t)W + lane];
        if (me == 0 && lane == 0 && updates < st.trace_cap) {
          st.trace_act[updates] = d.action;
          st.trace_idx[updates] = (int32_t)d.i;
        }
      }
      if constexpr (MULTI) {
        if (lane == 0) dec = d;
      }
    }
    __syncthreads();  // orders the LDS writes of pi_sh (and dec) before the reads below
    if constexpr (MULTI) d = dec;
    if (d.action != 1 && d.action != 2) {
      status = d.action == 0 ? 0 : (d.action == 3 ? 1 : -5);
      break;
    }
    ++updates;
    r = rec_empty<T>();
    float pir[kReg];
    if constexpr (MM > 0) {
#pragma unroll
      for (int e = 0; e < kReg; ++e) pir[e] = pi_sh[e];
    }
#pragma unroll
    for (int k = 0; k < PT; ++k) {
      if (jj[k] < j1) {
        T kv;
        if constexpr (MM > 0) {
          kv = kfk_regs<MM>(pjr[k], pir, st.half_g);
        } else {
          const float* pj = st.p_in_lds ? pslice + (jj[k] - j0) * (int64_t)W : st.P + jj[k] * (int64_t)W;
          kv = kfk_pair(pj, pi_sh, M, st.D, st.half_g);
        }
        F[k] = axpy_rn(d.dalpha, kv, F[k]);
        if (jj[k] == d.i) a[k] = (d.action == 1) ? a[k] + d.dalpha : (T)0;  // Eq. 7 / removal
        point_record(r, jj[k], y[k], F[k], a[k]);
      }
    }
    if constexpr (!kKeys) r = wave_allreduce(r);
    if constexpr (!MULTI) __syncthreads();  // pi_sh is rewritten in the next iteration
  }
#pragma unroll
  for (int k = 0; k < PT; ++k)
    if (jj[k] < j1) {
      st.F[jj[k]] = F[k];
      st.alpha[jj[k]] = a[k];
    }
  if (me == 0 && threadIdx.x == 0) {
    out[0] = updates;
    out[1] = status;
  }
}

__global__ void k_train_init(unsigned long long* words, int64_t nwords, int64_t* out) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < nwords) words[i] = 0ull;
  if (blockIdx.x == 0 && threadIdx.x < 2) out[threadIdx.x] = 0;
}

// removeNonsupportPoints: stable compaction of the indices with alpha != 0.
template <typename T>
__global__ void __launch_bounds__(1024) k_compact(const T* __restrict__ alpha, int64_t N, int32_t* __restrict__ idx,
                                                  int64_t* __restrict__ count) {
  __shared__ int wsum[16];
  __shared__ int64_t base;
  if (threadIdx.x == 0) base = 0;
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int64_t start = 0; start < N; start += 1024) {
    const int64_t j = start + threadIdx.x;
    const int flag = (j < N && alpha[j] != (T)0) ? 1 : 0;
    // inclusive scan within the wave
    int v = flag;
    for (int off = 1; off < 64; off <<= 1) {
      int o = __shfl_up(v, off);
      if (lane >= off) v += o;
    }
    if (lane == 63) wsum[wave] = v;
    __syncthreads();
    int before = 0;
    for (int w = 0; w < wave; ++w) before += wsum[w];
    if (flag) idx[base + before + v - 1] = (int32_t)j;
    __syncthreads();
    if (threadIdx.x == 0) {
      int tot = 0;
      for (int w = 0; w < 16; ++w) tot += wsum[w];
      base += tot;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) *count = base;
}

template <typename T, int MM, bool MULTI>
static const void* wave_kernel_mm(int PT) {
  if constexpr (MULTI && sizeof(T) == 8) {
    return reinterpret_cast<const void*>(k_train_wave<T, 1, MM, true>);  // FP64: one point per lane only
  } else if constexpr (MULTI) {
    switch (PT) {
      case 1: return reinterpret_cast<const void*>(k_train_wave<T, 1, MM, true>);
      case 2: return reinterpret_cast<const void*>(k_train_wave<T, 2, MM, true>);
      default: return reinterpret_cast<const void*>(k_train_wave<T, kMultiMaxPT, MM, true>);
    }
  } else {
    switch (PT) {
      case 1: return reinterpret_cast<const void*>(k_train_wave<T, 1, MM, false>);
      case 2: return reinterpret_cast<const void*>(k_train_wave<T, 2, MM, false>);
      case 4: return reinterpret_cast<const void*>(k_train_wave<T, 4, MM, false>);
      default:
        // coordinates stay in registers only up to 4 points per lane (the launch shapes never ask for more)
        if constexpr (MM > 0) return nullptr;
        else return PT == 8 ? reinterpret_cast<const void*>(k_train_wave<T, 8, 0, false>)
                            : reinterpret_cast<const void*>(k_train_wave<T, 16, 0, false>);
    }
  }
}

template <typename T>
static const void* wave_kernel(int PT, int mm, bool multi) {
  if (multi) {
    if (mm == 4) return wave_kernel_mm<T, 4, true>(PT);
    if (mm == 8) return wave_kernel_mm<T, 8, true>(PT);
    return wave_kernel_mm<T, 0, true>(PT);
  }
  if (mm == 4) return wave_kernel_mm<T, 4, false>(PT);
  if (mm == 8) return wave_kernel_mm<T, 8, false>(PT);
  return wave_kernel_mm<T, 0, false>(PT);
}

// Launch shape of the wave form for one training set of N points. Several
// waves per workgroup (nw > 1): one point per lane; a set that fits one
// workgroup of the largest size runs in one (no record exchange), else the
// waves double from nw up to 16 (8 in FP64) while the grid exceeds `cap`
// workgroups (more waves spread a
// workgroup's column over its CU's SIMDs; a workgroup holds at most 1,024
// points in this form whatever the split between waves and points per lane,
// so more points per lane would only lengthen every wave's column). Single-wave
// workgroups (nw = 1): PT points per lane, doubling up to 16 while the grid
// exceeds `cap`. Control points in registers for chains of 4 or 8 points (up
// to 4 points per lane), else in LDS when the slice fits in 48 KB. Returns
// false when the grid exceeds the form's limits or is not resident.
template <typename T>
static bool wave_shape(int64_t N, int M, int D, int nw, int64_t cap, int ncu, const void** kfn, int64_t* G,
                       int64_t* chunk, size_t* lds_bytes, int* threads) {
  const bool multi = nw > 1;
  auto groups = [&](int w, int pt) { return (N + 64ll * w * pt - 1) / (64ll * w * pt); };
  int PT = 1, waves = multi ? nw : 1;
  // FP64 workgroups stop at 8 waves (512 threads leave its register-held coordinates room without spills)
  const int max_waves = sizeof(T) == 8 ? 8 : 16;
  if (multi && waves > max_waves) waves = max_waves;
  // a set that fits one workgroup of the largest size (one point per lane) runs in one: the kernel then
  // skips the record exchange
  if (multi && groups(waves, 1) > 1 && groups(max_waves, 1) == 1 && tune_get("train.single_group") == 1) {
    waves = max_waves;
  } else if (multi) {
    while (waves < max_waves && groups(waves, PT) > cap) waves *= 2;
  } else {
    while (PT < 16 && groups(waves, PT) > cap) PT *= 2;
  }
  const int nt = 64 * waves;
  *chunk = (int64_t)nt * PT;
  *G = (N + *chunk - 1) / *chunk;
  if (*G > (int64_t)(multi ? kMultiChunks<T> : kWaveChunks) * 64) return false;
  const int mm = (D == 3 && PT <= 4 && (M == 4 || M == 8)) ? M : 0;
  *kfn = wave_kernel<T>(PT, mm, multi);
  if (*kfn == nullptr) return false;
  *lds_bytes = mm ? 0 : (size_t)*chunk * M * D * sizeof(float);
  if (*lds_bytes > 48 * 1024) *lds_bytes = 0;
  *threads = nt;
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, *kfn, nt, *lds_bytes) != hipSuccess) return false;
  return per_cu >= 1 && *G <= (int64_t)per_cu * ncu;
}

// Host validation shared by the points and configuration forms (before any HIP call).
template <typename T>
static fastron_status check_train_args(const int8_t* y, int64_t N, int32_t M, int32_t D, T gamma, T beta,
                                       int64_t iter_max, int64_t s_max, const T* alpha, const T* F,
                                       const int32_t* support_idx, const int64_t* n_support, const int64_t* updates,
                                       const int32_t* trace_action, const int32_t* trace_index, int64_t trace_cap) {
  FASTRON_CHECK(N >= 1 && N < INT32_MAX, "N = %lld outside [1, 2^31)", (long long)N);
  FASTRON_CHECK(M >= 1 && M <= FASTRON_MAX_POINTS, "M = %d outside [1, %d]", M, FASTRON_MAX_POINTS);
  FASTRON_CHECK(D >= 1 && M * D <= 3 * FASTRON_MAX_POINTS, "%d points of %d coordinates exceed %d floats", M, D,
                3 * FASTRON_MAX_POINTS);
  FASTRON_CHECK(y && alpha && F && support_idx, "y, alpha, F and support_idx must be non-NULL");
  FASTRON_CHECK(n_support && updates, "n_support and updates must be non-NULL host pointers");
  FASTRON_CHECK(std::isfinite((double)gamma) && gamma > 0, "gamma must be finite and > 0");
  FASTRON_CHECK(std::isfinite((double)beta) && beta >= 1, "beta must be >= 1 (Eq. 5)");
  FASTRON_CHECK(iter_max >= 0, "iter_max < 0");
  FASTRON_CHECK(s_max >= 1, "s_max must be >= 1");
  FASTRON_CHECK(trace_cap >= 0 && (trace_cap == 0 || (trace_action && trace_index)),
                "trace arrays must be non-NULL when trace_cap > 0");
  return FASTRON_OK;
}

template <typename T>
static fastron_status train_impl(const float* P, const int8_t* y, int64_t N, int32_t M, int32_t D, T gamma, T beta,
                                 int64_t iter_max, int64_t s_max, T* alpha, T* F, int32_t* support_idx,
                                 int64_t* n_support, int64_t* updates, int32_t* trace_action, int32_t* trace_index,
                                 int64_t trace_cap, void* stream) {
  clear_error();
  FASTRON_CHECK(P != nullptr, "P is NULL");
  fastron_status cs = check_train_args<T>(y, N, M, D, gamma, beta, iter_max, s_max, alpha, F, support_idx, n_support,
                                          updates, trace_action, trace_index, trace_cap);
  if (cs != FASTRON_OK) return cs;
  hipStream_t s = as_stream(stream);
  int dev = 0;
  FASTRON_HIP(hipGetDevice(&dev));
  int ncu = 0, coop = 0;
  FASTRON_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
  FASTRON_HIP(hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev));
  if (!coop) return fail(FASTRON_EUNSUPPORTED, "device does not support cooperative launches");
  // Launch shape. Default: the wave form with "train.waves" waves per
  // workgroup and at most "train.wave_groups" workgroups (see wave_shape),
  // falling back to single-wave workgroups when that grid does not fit.
  // Otherwise, or with "train.kernel" = 0: the slice kernel, a slice per
  // workgroup and at most one workgroup per CU, each thread holding PT points.
  int threads = 64;
  int64_t G = 0, chunk = 0;
  int PT = 1;
  const void* kfn = nullptr;
  size_t lds_bytes = 0;
  int per_cu = 0;
  if (tune_get("train.kernel") == 1) {
    const int64_t cap = tune_get("train.wave_groups");
    const int nw = (int)tune_get("train.waves");
    if (!wave_shape<T>(N, M, D, nw, cap, ncu, &kfn, &G, &chunk, &lds_bytes, &threads) &&
        (nw == 1 || !wave_shape<T>(N, M, D, 1, cap, ncu, &kfn, &G, &chunk, &lds_bytes, &threads)))
      kfn = nullptr;
  }
  if (kfn == nullptr) {
    threads = (int)tune_get("train.threads");
    G = tune_get("train.blocks");
    if (G <= 0) G = (N + 2 * threads - 1) / (2 * threads);  // about two points per thread
    if (G > ncu) G = ncu;
    if (G < 1) G = 1;
    chunk = (N + G - 1) / G;
    PT = 1;
    while ((int64_t)PT * threads < chunk) PT *= 2;
    if (PT > 16)
      return fail(FASTRON_EUNSUPPORTED, "N = %lld exceeds %lld training points (16 per thread on %d CUs)",
                  (long long)N, (long long)16 * threads * ncu, ncu);
    G = (N + chunk - 1) / chunk;
    switch (PT) {
      case 1: kfn = reinterpret_cast<const void*>(k_train<T, 1>); break;
      case 2: kfn = reinterpret_cast<const void*>(k_train<T, 2>); break;
      case 4: kfn = reinterpret_cast<const void*>(k_train<T, 4>); break;
      case 8: kfn = reinterpret_cast<const void*>(k_train<T, 8>); break;
      default: kfn = reinterpret_cast<const void*>(k_train<T, 16>); break;
    }
    // stage each slice's control points in LDS when they fit (48 KB budget)
    lds_bytes = (size_t)chunk * M * D * sizeof(float);
    if (lds_bytes > 48 * 1024) lds_bytes = 0;
    FASTRON_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kfn, threads, lds_bytes));
    if (per_cu < 1) return fail(FASTRON_EUNSUPPORTED, "training kernel cannot be resident with %d threads", threads);
  }
  const size_t rec_bytes = ((sizeof(unsigned long long) * 2 * (size_t)G * RecWords<T>::K + 255) / 256) * 256;
  char* ws = nullptr;
  FASTRON_HIP(hipMallocAsync(reinterpret_cast<void**>(&ws), rec_bytes + 256, s));
  Rec<T>* rec = reinterpret_cast<Rec<T>*>(ws);  // reinterpreted as record words by the kernel
  int64_t* out = reinterpret_cast<int64_t*>(ws + rec_bytes);
  int64_t* cnt = reinterpret_cast<int64_t*>(ws + rec_bytes + 64);
  hipLaunchKernelGGL(k_train_init, dim3((unsigned)((rec_bytes / 8 + 255) / 256)), dim3(256), 0, s,
                     reinterpret_cast<unsigned long long*>(ws), (int64_t)(rec_bytes / 8), out);
  fastron_status rs = FASTRON_OK;
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) {
    TrainState<T> st;
    st.P = P;
    st.y = y;
    st.alpha = alpha;
    st.F = F;
    st.rec = rec;
    st.out = out;
    st.trace_act = trace_action;
    st.trace_idx = trace_index;
    st.trace_cap = trace_cap;
    st.N = N;
    st.iter_max = iter_max;
    st.s_max = s_max;
    st.half_g = gamma / (T)2;
    st.beta = beta;
    st.M = M;
    st.D = D;
    st.chunk = (int)chunk;
    st.timeout = 400000000ll;  // 4 s at 100 MHz
    st.poll_delay = (int)tune_get("train.poll_delay");
    st.p_in_lds = lds_bytes > 0 ? 1 : 0;
    st.env_of = nullptr;
    st.env_wg0 = nullptr;
    st.env_off = nullptr;
    void* args[] = {&st};
    e = hipLaunchCooperativeKernel(kfn, dim3((unsigned)G), dim3((unsigned)threads), args, lds_bytes, s);
  }
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_compact<T>, dim3(1), dim3(1024), 0, s, alpha, N, support_idx, cnt);
    e = hipGetLastError();
  }
  int64_t host[3] = {0, 0, 0};
  if (e == hipSuccess) e = hipMemcpyAsync(host, out, 2 * sizeof(int64_t), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipMemcpyAsync(host + 2, cnt, sizeof(int64_t), hipMemcpyDeviceToHost, s);
  hipError_t ef = hipFreeAsync(ws, s);
  if (e == hipSuccess) e = ef;
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return fail(FASTRON_EHIP, "training launch failed: %s", hipGetErrorString(e));
  *updates = host[0];
  *n_support = host[2];
  if (host[1] == -5)
    return fail(FASTRON_EDEVICE, "record exchange timed out after %lld updates", (long long)host[0]);
  rs = host[1] == 0 ? FASTRON_OK : FASTRON_NOT_CONVERGED;
  return rs;
}

// Several independent training sets in one cooperative launch of the wave
// form: set e gets ceil(N_e / chunk) workgroups, its own records and its own
// exchange, so the sets advance concurrently.
static fastron_status train_batch_impl(const float* P, const int8_t* y, int32_t E, const int64_t* offsets, int32_t M,
                                       float gamma, float beta, int64_t iter_max, int64_t s_max, float* alpha, float* F,
                                       int32_t* support_idx, int64_t* n_support, int64_t* updates, void* stream) {
  clear_error();
  FASTRON_CHECK(E >= 1 && E <= 4096, "E = %d outside [1, 4096]", E);
  FASTRON_CHECK(offsets != nullptr, "offsets must be a non-NULL host array");
  FASTRON_CHECK(offsets[0] == 0, "offsets must start at 0");
  for (int e = 0; e < E; ++e)
    FASTRON_CHECK(offsets[e + 1] > offsets[e], "training set %d is empty or offsets decrease", e);
  const int64_t N = offsets[E];
  FASTRON_CHECK(N < INT32_MAX, "N = %lld outside [1, 2^31)", (long long)N);
  FASTRON_CHECK(M >= 1 && M <= FASTRON_MAX_POINTS, "M = %d outside [1, %d]", M, FASTRON_MAX_POINTS);
  FASTRON_CHECK(P && y && alpha && F && support_idx, "P, y, alpha, F and support_idx must be non-NULL");
  FASTRON_CHECK(n_support && updates, "n_support and updates must be non-NULL host arrays");
  FASTRON_CHECK(std::isfinite(gamma) && gamma > 0.f, "gamma must be finite and > 0");
  FASTRON_CHECK(std::isfinite(beta) && beta >= 1.f, "beta must be >= 1 (Eq. 5)");
  FASTRON_CHECK(iter_max >= 0, "iter_max < 0");
  FASTRON_CHECK(s_max >= 1, "s_max must be >= 1");
  hipStream_t s = as_stream(stream);
  int dev = 0, ncu = 0, coop = 0;
  FASTRON_HIP(hipGetDevice(&dev));
  FASTRON_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
  FASTRON_HIP(hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev));
  if (!coop) return fail(FASTRON_EUNSUPPORTED, "device does not support cooperative launches");
  // Launch shape: the smallest PT whose grid fits the cap per set and the
  // resident capacity in total, first with "train.waves" waves per workgroup
  // (at most 16 / PT, PT <= kMultiMaxPT), then with single-wave workgroups.
  const int64_t cap = tune_get("train.wave_groups");
  const int nw_tune = (int)tune_get("train.waves");
  int PT = 1, threads = 64;
  const void* kfn = nullptr;
  int64_t G = 0;
  size_t lds_bytes = 0;
  for (int multi = nw_tune > 1 ? 1 : 0; multi >= 0 && kfn == nullptr; --multi) {
    const int pt_max = multi ? kMultiMaxPT : 16;
    for (PT = 1; PT <= pt_max; PT *= 2) {
      const int nw = multi ? (nw_tune < 16 / PT ? nw_tune : 16 / PT) : 1;
      const int64_t chunk_try = 64ll * nw * PT;
      int64_t total = 0, largest = 0;
      for (int e = 0; e < E; ++e) {
        const int64_t ge = (offsets[e + 1] - offsets[e] + chunk_try - 1) / chunk_try;
        total += ge;
        largest = ge > largest ? ge : largest;
      }
      if (largest > cap && PT < pt_max) continue;
      if (largest > (int64_t)(multi ? kMultiChunks<float> : kWaveChunks) * 64) continue;
      const int mm = (PT <= 4 && (M == 4 || M == 8)) ? M : 0;
      const void* fn = wave_kernel<float>(PT, mm, multi == 1);
      if (fn == nullptr) continue;
      size_t lds = mm ? 0 : (size_t)chunk_try * 3 * M * sizeof(float);
      if (lds > 48 * 1024) lds = 0;
      int per_cu = 0;
      FASTRON_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, 64 * nw, lds));
      if (per_cu >= 1 && total <= (int64_t)per_cu * ncu) {
        kfn = fn;
        G = total;
        lds_bytes = lds;
        threads = 64 * nw;
        break;
      }
    }
  }
  if (kfn == nullptr) return fail(FASTRON_EUNSUPPORTED, "training sets too large for one resident launch");
  const int64_t chunk = (int64_t)threads * PT;
  std::vector<int32_t> env_of((size_t)G), env_wg0((size_t)E + 1);
  env_wg0[0] = 0;
  for (int e = 0; e < E; ++e) {
    const int64_t ge = (offsets[e + 1] - offsets[e] + chunk - 1) / chunk;
    env_wg0[e + 1] = env_wg0[e] + (int32_t)ge;
    for (int64_t w = env_wg0[e]; w < env_wg0[e + 1]; ++w) env_of[(size_t)w] = e;
  }
  constexpr int K = RecWords<float>::K;
  const size_t rec_bytes = ((sizeof(unsigned long long) * 2 * (size_t)G * K + 255) / 256) * 256;
  const size_t tab_bytes = ((sizeof(int32_t) * ((size_t)G + E + 1) + sizeof(int64_t) * (E + 1) + 255) / 256) * 256;
  const size_t out_bytes = ((sizeof(int64_t) * 3 * (size_t)E + 255) / 256) * 256;
  char* ws = nullptr;
  FASTRON_HIP(hipMallocAsync(reinterpret_cast<void**>(&ws), rec_bytes + tab_bytes + out_bytes, s));
  int32_t* d_env_of = reinterpret_cast<int32_t*>(ws + rec_bytes);
  int32_t* d_env_wg0 = d_env_of + G;
  int64_t* d_env_off = reinterpret_cast<int64_t*>(ws + rec_bytes + tab_bytes - sizeof(int64_t) * (E + 1));
  int64_t* out = reinterpret_cast<int64_t*>(ws + rec_bytes + tab_bytes);  // [E][2], then counts [E]
  int64_t* cnt = out + 2 * E;
  hipError_t e = hipMemcpyAsync(d_env_of, env_of.data(), sizeof(int32_t) * G, hipMemcpyHostToDevice, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(d_env_wg0, env_wg0.data(), sizeof(int32_t) * (E + 1), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(d_env_off, offsets, sizeof(int64_t) * (E + 1), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_train_init, dim3((unsigned)((rec_bytes / 8 + 255) / 256)), dim3(256), 0, s,
                       reinterpret_cast<unsigned long long*>(ws), (int64_t)(rec_bytes / 8), out);
    e = hipGetLastError();
  }
  if (e == hipSuccess) {
    TrainState<float> st;
    st.P = P;
    st.y = y;
    st.alpha = alpha;
    st.F = F;
    st.rec = reinterpret_cast<Rec<float>*>(ws);
    st.out = out;
    st.trace_act = nullptr;
    st.trace_idx = nullptr;
    st.trace_cap = 0;
    st.N = N;
    st.iter_max = iter_max;
    st.s_max = s_max;
    st.half_g = gamma / 2.0f;
    st.beta = beta;
    st.M = M;
    st.D = 3;
    st.chunk = (int)chunk;
    st.timeout = 400000000ll;  // 4 s at 100 MHz
    st.poll_delay = (int)tune_get("train.poll_delay");
    st.p_in_lds = lds_bytes > 0 ? 1 : 0;
    st.env_of = d_env_of;
    st.env_wg0 = d_env_wg0;
    st.env_off = d_env_off;
    void* args[] = {&st};
    e = hipLaunchCooperativeKernel(kfn, dim3((unsigned)G), dim3((unsigned)threads), args, lds_bytes, s);
  }
  for (int k = 0; k < E && e == hipSuccess; ++k) {
    hipLaunchKernelGGL(k_compact<float>, dim3(1), dim3(1024), 0, s, alpha + offsets[k], offsets[k + 1] - offsets[k],
                       support_idx + offsets[k], cnt + k);
    e = hipGetLastError();
  }
  std::vector<int64_t> host((size_t)3 * E, 0);
  if (e == hipSuccess) e = hipMemcpyAsync(host.data(), out, sizeof(int64_t) * 3 * E, hipMemcpyDeviceToHost, s);
  const hipError_t ef = hipFreeAsync(ws, s);
  if (e == hipSuccess) e = ef;
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return fail(FASTRON_EHIP, "batched training failed: %s", hipGetErrorString(e));
  bool all_converged = true;
  for (int k = 0; k < E; ++k) {
    updates[k] = host[2 * k];
    n_support[k] = host[2 * E + k];
    if (host[2 * k + 1] == -5)
      return fail(FASTRON_EDEVICE, "record exchange of training set %d timed out after %lld updates", k,
                  (long long)host[2 * k]);
    if (host[2 * k + 1] != 0) all_converged = false;
  }
  return all_converged ? FASTRON_OK : FASTRON_NOT_CONVERGED;
}

// Configuration forms: Algorithm 1's input is a dataset of configurations
// (Section III-B). Their control points (a1, one FK per configuration) go
// into stream-ordered scratch of N x M x 3 floats, and the points form runs on
// them: the same kernels, so the two forms give bit-identical results.
template <typename T>
static fastron_status train_configs(const fastron_chain* chain, const fastron_cpoints* cp, const float* X,
                                    const int8_t* y, int64_t N, T gamma, T beta, int64_t iter_max, int64_t s_max,
                                    T* alpha, T* F, int32_t* support_idx, int64_t* n_support, int64_t* updates,
                                    int32_t* trace_action, int32_t* trace_index, int64_t trace_cap, void* stream) {
  clear_error();
  ChainArgs c;
  fastron_status st = pack_chain(chain, cp, &c, true);
  if (st != FASTRON_OK) return st;
  FASTRON_CHECK(X != nullptr, "X is NULL");
  st = check_train_args<T>(y, N, c.M, 3, gamma, beta, iter_max, s_max, alpha, F, support_idx, n_support, updates,
                           trace_action, trace_index, trace_cap);
  if (st != FASTRON_OK) return st;
  hipStream_t s = as_stream(stream);
  float* P = nullptr;
  FASTRON_HIP(hipMallocAsync(reinterpret_cast<void**>(&P), (size_t)N * c.M * 3 * sizeof(float), s));
  st = fastron_fk_points(chain, cp, X, N, P, stream);
  if (st == FASTRON_OK)
    st = train_impl<T>(P, y, N, c.M, 3, gamma, beta, iter_max, s_max, alpha, F, support_idx, n_support, updates,
                       trace_action, trace_index, trace_cap, stream);
  const hipError_t ef = hipFreeAsync(P, s);
  if (st != FASTRON_OK && st != FASTRON_NOT_CONVERGED) return st;
  if (ef != hipSuccess) return fail(FASTRON_EHIP, "hipFreeAsync failed: %s", hipGetErrorString(ef));
  return st;
}

}  // namespace fastron

using namespace fastron;

extern "C" {

fastron_status fastron_gram_update(const fastron_chain* chain, const fastron_cpoints* cp, const float* X, int64_t N,
                                   float gamma, int64_t i, float delta_alpha, float* F, float* kcol, void* stream) {
  clear_error();
  ChainArgs c;
  fastron_status st = pack_chain(chain, cp, &c, true);
  if (st != FASTRON_OK) return st;
  FASTRON_CHECK(N >= 1, "N = %lld < 1", (long long)N);
  FASTRON_CHECK(i >= 0 && i < N, "i = %lld outside [0, N)", (long long)i);
  FASTRON_CHECK(X != nullptr, "X is NULL");
  FASTRON_CHECK(F != nullptr || kcol != nullptr, "F and kcol are both NULL");
  FASTRON_CHECK(std::isfinite(gamma) && gamma > 0.f, "gamma must be finite and > 0");
  FASTRON_CHECK(std::isfinite(delta_alpha), "delta_alpha must be finite");
  FASTRON_CHECK((N + 255) / 256 <= INT32_MAX, "N too large");
  hipStream_t s = as_stream(stream);
  float* P = nullptr;
  FASTRON_HIP(hipMallocAsync(reinterpret_cast<void**>(&P), (size_t)N * c.M * 3 * sizeof(float), s));
  st = fastron_fk_points(chain, cp, X, N, P, stream);
  if (st == FASTRON_OK) st = fastron_gram_update_points(P, N, c.M, gamma, i, delta_alpha, F, kcol, stream);
  const hipError_t ef = hipFreeAsync(P, s);
  if (st != FASTRON_OK) return st;
  if (ef != hipSuccess) return fail(FASTRON_EHIP, "hipFreeAsync failed: %s", hipGetErrorString(ef));
  return FASTRON_OK;
}

fastron_status fastron_gram_update_points(const float* P, int64_t N, int32_t M, float gamma, int64_t i,
                                          float delta_alpha, float* F, float* kcol, void* stream) {
  clear_error();
  FASTRON_CHECK(N >= 1, "N = %lld < 1", (long long)N);
  FASTRON_CHECK(M >= 1 && M <= FASTRON_MAX_POINTS, "M = %d outside [1, %d]", M, FASTRON_MAX_POINTS);
  FASTRON_CHECK(i >= 0 && i < N, "i = %lld outside [0, N)", (long long)i);
  FASTRON_CHECK(P != nullptr, "P is NULL");
  FASTRON_CHECK(F != nullptr || kcol != nullptr, "F and kcol are both NULL");
  FASTRON_CHECK(std::isfinite(gamma) && gamma > 0.f, "gamma must be finite and > 0");
  FASTRON_CHECK(std::isfinite(delta_alpha), "delta_alpha must be finite");
  const int64_t blocks = (N + 255) / 256;
  FASTRON_CHECK(blocks <= INT32_MAX, "N too large");
  hipLaunchKernelGGL(k_gram_update, dim3((unsigned)blocks), dim3(256), 0, as_stream(stream), P, N, M, 0.5f * gamma,
                     i, delta_alpha, F, kcol);
  FASTRON_HIP(hipGetLastError());
  return FASTRON_OK;
}

fastron_status fastron_train(const fastron_chain* chain, const fastron_cpoints* cp, const float* X, const int8_t* y,
                             int64_t N, float gamma, float beta, int64_t iter_max, int64_t s_max, float* alpha,
                             float* F, int32_t* support_idx, int64_t* n_support, int64_t* updates,
                             int32_t* trace_action, int32_t* trace_index, int64_t trace_cap, void* stream) {
  return train_configs<float>(chain, cp, X, y, N, gamma, beta, iter_max, s_max, alpha, F, support_idx, n_support,
                              updates, trace_action, trace_index, trace_cap, stream);
}

fastron_status fastron_train_f64(const fastron_chain* chain, const fastron_cpoints* cp, const float* X,
                                 const int8_t* y, int64_t N, double gamma, double beta, int64_t iter_max,
                                 int64_t s_max, double* alpha, double* F, int32_t* support_idx, int64_t* n_support,
                                 int64_t* updates, int32_t* trace_action, int32_t* trace_index, int64_t trace_cap,
                                 void* stream) {
  return train_configs<double>(chain, cp, X, y, N, gamma, beta, iter_max, s_max, alpha, F, support_idx, n_support,
                               updates, trace_action, trace_index, trace_cap, stream);
}

fastron_status fastron_train_points(const float* P, const int8_t* y, int64_t N, int32_t M, float gamma, float beta,
                                    int64_t iter_max, int64_t s_max, float* alpha, float* F, int32_t* support_idx,
                                    int64_t* n_support, int64_t* updates, int32_t* trace_action,
                                    int32_t* trace_index, int64_t trace_cap, void* stream) {
  return train_impl<float>(P, y, N, M, 3, gamma, beta, iter_max, s_max, alpha, F, support_idx, n_support, updates,
                           trace_action, trace_index, trace_cap, stream);
}

fastron_status fastron_train_batch(const float* P, const int8_t* y, int32_t E, const int64_t* offsets, int32_t M,
                                   float gamma, float beta, int64_t iter_max, int64_t s_max, float* alpha, float* F,
                                   int32_t* support_idx, int64_t* n_support, int64_t* updates, void* stream) {
  return train_batch_impl(P, y, E, offsets, M, gamma, beta, iter_max, s_max, alpha, F, support_idx, n_support, updates,
                          stream);
}

fastron_status fastron_train_points_f64(const float* P, const int8_t* y, int64_t N, int32_t M, double gamma,
                                        double beta, int64_t iter_max, int64_t s_max, double* alpha, double* F,
                                        int32_t* support_idx, int64_t* n_support, int64_t* updates,
                                        int32_t* trace_action, int32_t* trace_index, int64_t trace_cap,
                                        void* stream) {
  return train_impl<double>(P, y, N, M, 3, gamma, beta, iter_max, s_max, alpha, F, support_idx, n_support, updates,
                            trace_action, trace_index, trace_cap, stream);
}

fastron_status fastron_rbf_train(const float* X, const int8_t* y, int64_t N, int32_t n, float gamma, float beta,
                                 int64_t iter_max, int64_t s_max, float* alpha, float* F, int32_t* support_idx,
                                 int64_t* n_support, int64_t* updates, void* stream) {
  clear_error();
  FASTRON_CHECK(n >= 1 && n <= FASTRON_MAX_JOINTS, "n = %d outside [1, %d]", n, FASTRON_MAX_JOINTS);
  return train_impl<float>(X, y, N, 1, n, gamma, beta, iter_max, s_max, alpha, F, support_idx, n_support, updates,
                           nullptr, nullptr, 0, stream);
}

fastron_status fastron_rbf_train_f64(const float* X, const int8_t* y, int64_t N, int32_t n, double gamma,
                                     double beta, int64_t iter_max, int64_t s_max, double* alpha, double* F,
                                     int32_t* support_idx, int64_t* n_support, int64_t* updates,
                                     int32_t* trace_action, int32_t* trace_index, int64_t trace_cap, void* stream) {
  clear_error();
  FASTRON_CHECK(n >= 1 && n <= FASTRON_MAX_JOINTS, "n = %d outside [1, %d]", n, FASTRON_MAX_JOINTS);
  return train_impl<double>(X, y, N, 1, n, gamma, beta, iter_max, s_max, alpha, F, support_idx, n_support, updates,
                            trace_action, trace_index, trace_cap, stream);
}

}  // extern "C"
