/*
 * FP64 CPU oracle for Fastron with the forward-kinematics (FK) kernel
 * (Das & Yip, "Forward Kinematics Kernel for Improved Proxy Collision Checking").
 *
 * TEST INFRASTRUCTURE ONLY. This file is the slow, plain, obviously-correct
 * reference that the GPU library is checked against. Only the test suite, the
 * smoke check and the CPU-baseline leg of the benchmark may load it. It shares
 * no code, header, table or helper with the GPU library, and the GPU library
 * never calls it.
 *
 * Everything is IEEE double precision, evaluated in the order the paper's
 * definitions are written. Inputs that arrive as float32 are upcast exactly by
 * the caller. OpenMP is used only across independent queries / columns entries;
 * it never changes the arithmetic of one result.
 *
 * Contents
 *   - D-H link transform                       (Section II-A, Eq. 1)
 *   - chain product and control points        (Section II-A, chain product, Eq. 2)
 *   - rational-quadratic kernel K_RQ           (Section II-B, Eq. 3)
 *   - FK kernel K_FK                           (Section III-A, Eq. 4)
 *   - Fastron score f(x) and its sign          (Section III-B, model definition)
 *   - Fastron model update, Algorithm 1        (Section III-B, Eq. 5-9, Algorithm 1)
 *   - loss L(alpha)                            (Section III-B, Eq. 5)
 *   - capsule-vs-axis-aligned-box labeller     (stands in for the geometric checker
 *                                                of Section IV; not part of the paper)
 */
#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------- */
/* Section II-A, Eq. 1: homogeneous transform of joint i in the frame of joint
 * i-1 under the standard D-H convention. Row-major 4x4. The matrix, not the
 * surrounding prose, decides the roles of a_i (x/y translation, multiplied by
 * cos/sin theta) and d_i (z translation).                                    */
void oracle_dh_link(double theta, double alpha, double a, double d, double A[16]) {
  double ct = cos(theta), st = sin(theta);
  double ca = cos(alpha), sa = sin(alpha);
  A[0] = ct;   A[1] = -ca * st; A[2] = sa * st;  A[3] = a * ct;
  A[4] = st;   A[5] = ca * ct;  A[6] = -sa * ct; A[7] = a * st;
  A[8] = 0.0;  A[9] = sa;       A[10] = ca;      A[11] = d;
  A[12] = 0.0; A[13] = 0.0;     A[14] = 0.0;     A[15] = 1.0;
}

static void mat4_mul(const double X[16], const double Y[16], double Z[16]) {
  for (int r = 0; r < 4; ++r)
    for (int c = 0; c < 4; ++c) {
      double s = 0.0;
      for (int k = 0; k < 4; ++k) s += X[4 * r + k] * Y[4 * k + c];
      Z[4 * r + c] = s;
    }
}

/* D-H table row layout used throughout the oracle: (a, alpha, d, theta, type)
 * per joint; type 0 = revolute (the joint variable is added to theta),
 * type 1 = prismatic (the joint variable is added to d). Section II-A states
 * that theta_i and d_i are the revolute and prismatic joint variables.       */
#define DH_COLS 5

/* Section II-A, chain product: wA_i = wA_0 * 0A_1 * ... * (i-1)A_i.
 * T receives n+1 row-major 4x4 matrices; T[0] = wA_0 (base, NULL = identity). */
void oracle_frames(int n, const double* dh, const double* base, const double* q, double* T) {
  double* T0 = T;
  for (int k = 0; k < 16; ++k) T0[k] = base ? base[k] : ((k % 5) == 0 ? 1.0 : 0.0);
  for (int i = 0; i < n; ++i) {
    const double* row = dh + DH_COLS * i;
    double a = row[0], alpha = row[1], d = row[2], theta = row[3];
    if ((int)row[4] == 0) theta += q[i]; else d += q[i];
    double A[16];
    oracle_dh_link(theta, alpha, a, d, A);
    mat4_mul(T + 16 * i, A, T + 16 * (i + 1));
  }
}

/* Eq. 2: FK_m(x) = pos(wA_{j_m} T_m). T_m is a static translation by
 * offset[m] (NULL = identity, the placement used in Section III-A), so
 * pos(wA T_m) = R * offset + p. P receives M x 3.                             */
void oracle_control_points(int n, const double* dh, const double* base, int M, const int* frame,
                           const double* offset, const double* q, double* P) {
  double* T = (double*)malloc(sizeof(double) * 16 * (size_t)(n + 1));
  oracle_frames(n, dh, base, q, T);
  for (int m = 0; m < M; ++m) {
    const double* A = T + 16 * frame[m];
    double Tm[16] = {1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1};
    if (offset) { Tm[3] = offset[3 * m]; Tm[7] = offset[3 * m + 1]; Tm[11] = offset[3 * m + 2]; }
    double AT[16];
    mat4_mul(A, Tm, AT);
    P[3 * m + 0] = AT[3];
    P[3 * m + 1] = AT[7];
    P[3 * m + 2] = AT[11];
  }
  free(T);
}

/* Section III-A, placement of control points: one point at each joint frame
 * origin, except that a revolute joint with a_i = d_i = 0 gets none, because
 * its origin always coincides with the preceding one. Frame i (1..n) is the
 * origin after D-H row i-1. With include_base, frame 0 (the base origin) is
 * listed first. Returns M; frame receives the kept frame indices in order.   */
int oracle_control_point_frames(int n, const double* dh, int include_base, int* frame) {
  int M = 0;
  if (include_base) frame[M++] = 0;
  for (int i = 1; i <= n; ++i) {
    const double* row = dh + DH_COLS * (i - 1);
    int revolute = (int)row[4] == 0;
    if (revolute && row[0] == 0.0 && row[2] == 0.0) continue;
    frame[M++] = i;
  }
  return M;
}

/* Batched control points for N configurations (q is N x n, P is N x M x 3). */
void oracle_control_points_batch(int n, const double* dh, const double* base, int M, const int* frame,
                                 const double* offset, int64_t N, const double* q, double* P) {
#pragma omp parallel for schedule(static)
  for (int64_t j = 0; j < N; ++j)
    oracle_control_points(n, dh, base, M, frame, offset, q + (size_t)n * j, P + (size_t)3 * M * j);
}

/* Section II-B, Eq. 3: second-order rational quadratic kernel
 * K_RQ(x, x') = (1 + gamma/2 * ||x - x'||^2)^(-2), with direct differences.  */
double oracle_k_rq(const double* x, const double* xp, int dim, double gamma) {
  double d2 = 0.0;
  for (int k = 0; k < dim; ++k) {
    double diff = x[k] - xp[k];
    d2 += diff * diff;
  }
  double base = 1.0 + 0.5 * gamma * d2;
  return 1.0 / (base * base);
}

/* Section III-A, Eq. 4: K(x, x') = (1/M) sum_m K_RQ(p_m(x), p_m(x')) over M
 * points of D coordinates each. D = 3 with the control points FK_m is the FK
 * kernel; M = 1 with the joint vector itself (D = n) is the rational
 * quadratic kernel on configurations, the baseline the paper compares with
 * (Section II-B, Eq. 3).                                                     */
double oracle_k_pts(int M, int D, const double* Px, const double* Pxp, double gamma) {
  double s = 0.0;
  for (int m = 0; m < M; ++m) s += oracle_k_rq(Px + (size_t)D * m, Pxp + (size_t)D * m, D, gamma);
  return s / (double)M;
}

/* The FK kernel of Eq. 4 on two M x 3 control-point sets. */
double oracle_k_fk(int M, const double* Px, const double* Pxp, double gamma) {
  return oracle_k_pts(M, 3, Px, Pxp, gamma);
}

/* Kernel matrix K_ij = K_FK(X_i, X_j) over N configurations given as control
 * points (Section II-B, kernel matrix definition). K is N x N row-major.      */
void oracle_gram_pts(int64_t N, int M, int D, const double* P, double gamma, double* K) {
  const size_t w = (size_t)D * M;
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < N; ++i)
    for (int64_t j = 0; j < N; ++j) K[i * N + j] = oracle_k_pts(M, D, P + w * i, P + w * j, gamma);
}
void oracle_gram(int64_t N, int M, const double* P, double gamma, double* K) { oracle_gram_pts(N, M, 3, P, gamma, K); }

/* Summand matrix K_m (the RQ matrix of control point m alone), Section III-A. */
void oracle_gram_summand(int64_t N, int M, const double* P, double gamma, int m, double* K) {
  for (int64_t i = 0; i < N; ++i)
    for (int64_t j = 0; j < N; ++j)
      K[i * N + j] = oracle_k_rq(P + (size_t)3 * M * i + 3 * m, P + (size_t)3 * M * j + 3 * m, 3, gamma);
}

/* Section III-B: Fastron model f(x) = sum_i K(S_i, x) alpha_i over the support
 * set, summed in support-index order. Support and query control points are
 * given (S x M x 3 and N x M x 3).                                           */
void oracle_score_pts(int M, int D, int64_t S, const double* Ps, const double* alpha, double gamma,
                      int64_t N, const double* Pq, double* f) {
  const size_t w = (size_t)D * M;
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t j = 0; j < N; ++j) {
    double acc = 0.0;
    for (int64_t i = 0; i < S; ++i) acc += oracle_k_pts(M, D, Ps + w * i, Pq + w * j, gamma) * alpha[i];
    f[j] = acc;
  }
}
void oracle_score_points(int M, int64_t S, const double* Ps, const double* alpha, double gamma,
                         int64_t N, const double* Pq, double* f) {
  oracle_score_pts(M, 3, S, Ps, alpha, gamma, N, Pq, f);
}

/* Score from joint configurations: FK of supports and queries (Eq. 2), then
 * the model sum above. sq is S x n, q is N x n.                               */
void oracle_score(int n, const double* dh, const double* base, int M, const int* frame,
                  const double* offset, int64_t S, const double* sq, const double* alpha, double gamma,
                  int64_t N, const double* q, double* f) {
  double* Ps = (double*)malloc(sizeof(double) * 3 * (size_t)M * (size_t)(S > 0 ? S : 1));
  for (int64_t i = 0; i < S; ++i)
    oracle_control_points(n, dh, base, M, frame, offset, sq + (size_t)n * i, Ps + (size_t)3 * M * i);
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t j = 0; j < N; ++j) {
    double Pq[3 * 64];
    oracle_control_points(n, dh, base, M, frame, offset, q + (size_t)n * j, Pq);
    double acc = 0.0;
    for (int64_t i = 0; i < S; ++i) acc += oracle_k_fk(M, Ps + (size_t)3 * M * i, Pq, gamma) * alpha[i];
    f[j] = acc;
  }
  free(Ps);
}

/* Section III-B, Eq. 5: L(alpha) = 1/2 alpha^T K alpha - y^T B alpha with
 * b_i = beta^(0.5 (y_i + 1)). Used only by invariant tests.                  */
double oracle_loss_pts(int64_t N, int M, int D, const double* P, const int* y, double gamma, double beta,
                       const double* alpha) {
  const size_t w = (size_t)D * M;
  double quad = 0.0, lin = 0.0;
  for (int64_t i = 0; i < N; ++i) {
    if (alpha[i] == 0.0) continue;
    for (int64_t j = 0; j < N; ++j) {
      if (alpha[j] == 0.0) continue;
      quad += alpha[i] * oracle_k_pts(M, D, P + w * i, P + w * j, gamma) * alpha[j];
    }
    lin += (double)y[i] * pow(beta, 0.5 * (y[i] + 1)) * alpha[i];
  }
  return 0.5 * quad - lin;
}
double oracle_loss(int64_t N, int M, const double* P, const int* y, double gamma, double beta,
                   const double* alpha) {
  return oracle_loss_pts(N, M, 3, P, y, gamma, beta, alpha);
}

/* Column i of the kernel matrix K, evaluated when an update needs it (the
 * lazy evaluation described in Section III-B).                              */
static void kernel_column(int64_t N, int M, int D, const double* P, double gamma, int64_t i, double* col) {
  const size_t w = (size_t)D * M;
#pragma omp parallel for schedule(static)
  for (int64_t j = 0; j < N; ++j) col[j] = oracle_k_pts(M, D, P + w * j, P + w * i, gamma);
}

/* Trace action codes for oracle_fastron_update.                            */
#define ACT_ADD 1
#define ACT_REMOVE 2

/* Index of the smallest margin y_j F_j (the first one among equal values),
 * -1 for an empty set; *m receives the margin.                              */
static int64_t smallest_margin(int64_t N, const int* y, const double* F, double* m) {
  int64_t best = -1;
  for (int64_t j = 0; j < N; ++j) {
    const double v = (double)y[j] * F[j];
    if (best < 0 || v < *m) {
      best = j;
      *m = v;
    }
  }
  return best;
}

/* Among the weighted points, the index of the largest y_j (F_j - alpha_j),
 * the margin point j keeps without its own term (K_jj = 1); the first one
 * among equal values, -1 when no point has a weight.                       */
static int64_t most_redundant(int64_t N, const int* y, const double* F, const double* alpha, double* v) {
  int64_t best = -1;
  for (int64_t j = 0; j < N; ++j) {
    if (alpha[j] == 0.0) continue;
    const double u = (double)y[j] * (F[j] - alpha[j]);
    if (best < 0 || u > *v) {
      best = j;
      *v = u;
    }
  }
  return best;
}

/*
 * Fastron model update (Section III-B, Algorithm 1) as greedy coordinate
 * descent on the weights alpha, keeping F = K alpha current so that y_j F_j
 * is point j's margin. Each update moves one weight alpha_i by delta and F by
 * delta times column i of K (Eq. 8), the column evaluated only then (the lazy
 * kernel evaluation of Section III-B). Which weight moves:
 *   - a correction, when the smallest margin is <= 0 (Eq. 9): that point
 *     (the first of equal margins) gets delta = b_i y_i - F_i, after which its
 *     margin is exactly b_i (Eq. 6-7; b_i = beta for y_i = +1 and 1 for
 *     y_i = -1, the conditional bias of Eq. 5); allowed while fewer than s_max
 *     points carry a weight, or when point i already does;
 *   - otherwise a pruning: among the weighted points, the one with the
 *     largest y_j (F_j - alpha_j), if that value is > 0 (the point stays
 *     correctly classified without its own term), loses its weight,
 *     delta = -alpha_i (the first of equal values);
 *   - if neither applies, the update has converged.
 * At most iter_max updates are made. The weights and F come in (zeros for a
 * fresh model, or a previous model with F = K alpha); afterwards the support
 * set is the weighted points in ascending index order.
 *
 * P holds the control points of the N training configurations (N x M x D),
 * y holds +1 (in collision) / -1 (free). Returns 0 on convergence, 1 when
 * iter_max updates were made first. *updates receives the number of updates.
 * Optional trace arrays (capacity trace_cap) receive, per update, the action
 * (1 correction, 2 pruning), the index and delta.                           */
int oracle_fastron_update_pts(int64_t N, int M, int D, const double* P, const int* y, double gamma, double beta,
                              int64_t iter_max, int64_t s_max, double* alpha, double* F, int64_t* updates,
                              int64_t* support_idx, int64_t* n_support, int64_t trace_cap, int* trace_act,
                              int64_t* trace_idx, double* trace_dalpha) {
  double* col = (double*)malloc(sizeof(double) * (size_t)(N > 0 ? N : 1));
  int64_t weighted = 0;
  for (int64_t j = 0; j < N; ++j) weighted += (alpha[j] != 0.0);
  int64_t done = 0;
  int converged = 0;
  while (done < iter_max) {
    int act = 0;
    int64_t i = -1;
    double delta = 0.0, m = 0.0;
    const int64_t w = smallest_margin(N, y, F, &m);
    if (w >= 0 && m <= 0.0 && (weighted < s_max || alpha[w] != 0.0)) {
      const double b = y[w] > 0 ? beta : 1.0;
      act = ACT_ADD;
      i = w;
      delta = b * (double)y[w] - F[w];
    } else {
      double v = 0.0;
      const int64_t r = most_redundant(N, y, F, alpha, &v);
      if (r >= 0 && v > 0.0) {
        act = ACT_REMOVE;
        i = r;
        delta = -alpha[r];
      }
    }
    if (!act) {
      converged = 1;
      break;
    }
    kernel_column(N, M, D, P, gamma, i, col);
    const int had_weight = alpha[i] != 0.0;
    alpha[i] += delta;
    for (int64_t j = 0; j < N; ++j) F[j] += delta * col[j];
    weighted += (alpha[i] != 0.0) - had_weight;
    if (done < trace_cap) {
      trace_act[done] = act;
      trace_idx[done] = i;
      trace_dalpha[done] = delta;
    }
    ++done;
  }
  int64_t ns = 0;
  for (int64_t j = 0; j < N; ++j)
    if (alpha[j] != 0.0) {
      if (support_idx) support_idx[ns] = j;
      ++ns;
    }
  if (n_support) *n_support = ns;
  if (updates) *updates = done;
  free(col);
  return converged ? 0 : 1;
}

int oracle_fastron_update(int64_t N, int M, const double* P, const int* y, double gamma, double beta,
                          int64_t iter_max, int64_t s_max, double* alpha, double* F, int64_t* updates,
                          int64_t* support_idx, int64_t* n_support, int64_t trace_cap, int* trace_act,
                          int64_t* trace_idx, double* trace_dalpha) {
  return oracle_fastron_update_pts(N, M, 3, P, y, gamma, beta, iter_max, s_max, alpha, F, updates, support_idx,
                                   n_support, trace_cap, trace_act, trace_idx, trace_dalpha);
}

/* ------------------------------------------------------------------------- */
/* Geometric labeller (stands in for the ground-truth checker of Section IV).
 * Link i of the arm is a capsule of radius r around the segment from the
 * origin of frame i-1 to the origin of frame i (i = 1..n); a zero-length link
 * is a sphere. Obstacles are axis-aligned boxes [lo, hi]. A configuration is
 * in collision (+1) iff some capsule touches some box: the exact distance
 * from the segment to the box is <= r. Self-collision and the ground are not
 * modelled.
 *
 * Exact segment-to-box distance: with P(t) = A + t (B - A), t in [0, 1],
 * g(t) = sum_k phi_k(P_k(t))^2, phi_k(u) = max(lo_k - u, 0, u - hi_k),
 * is convex and quadratic between the (at most six) parameters where some
 * P_k(t) crosses lo_k or hi_k. The minimum over [0, 1] is therefore attained
 * at an end point of such a piece or at the stationary point of the piece's
 * quadratic, clipped to the piece; all of these are evaluated.            */

static double box_dist2(const double p[3], const double lo[3], const double hi[3]) {
  double s = 0.0;
  for (int k = 0; k < 3; ++k) {
    double e = 0.0;
    if (p[k] < lo[k]) e = lo[k] - p[k];
    else if (p[k] > hi[k]) e = p[k] - hi[k];
    s += e * e;
  }
  return s;
}

static double seg_point_dist2(const double A[3], const double D[3], double t, const double lo[3],
                              const double hi[3]) {
  double p[3] = {A[0] + t * D[0], A[1] + t * D[1], A[2] + t * D[2]};
  return box_dist2(p, lo, hi);
}

static int cmp_dbl(const void* a, const void* b) {
  double x = *(const double*)a, y = *(const double*)b;
  return (x > y) - (x < y);
}

double oracle_segment_box_dist2(const double A[3], const double B[3], const double lo[3], const double hi[3]) {
  double D[3] = {B[0] - A[0], B[1] - A[1], B[2] - A[2]};
  double ts[8];
  int nt = 0;
  ts[nt++] = 0.0;
  ts[nt++] = 1.0;
  for (int k = 0; k < 3; ++k) {
    if (D[k] == 0.0) continue;
    double t0 = (lo[k] - A[k]) / D[k], t1 = (hi[k] - A[k]) / D[k];
    if (t0 > 0.0 && t0 < 1.0) ts[nt++] = t0;
    if (t1 > 0.0 && t1 < 1.0) ts[nt++] = t1;
  }
  qsort(ts, (size_t)nt, sizeof(double), cmp_dbl);
  double best = seg_point_dist2(A, D, 0.0, lo, hi);
  for (int s = 0; s + 1 < nt; ++s) {
    double ta = ts[s], tb = ts[s + 1];
    double e_a = seg_point_dist2(A, D, ta, lo, hi), e_b = seg_point_dist2(A, D, tb, lo, hi);
    if (e_a < best) best = e_a;
    if (e_b < best) best = e_b;
    if (tb <= ta) continue;
    /* On (ta, tb) every coordinate stays on one side of its slab: read the
     * side at the midpoint and minimise sum_k (c_k + D_k t)^2 over active k. */
    double tm = 0.5 * (ta + tb);
    double num = 0.0, den = 0.0;
    for (int k = 0; k < 3; ++k) {
      double u = A[k] + tm * D[k];
      double c;
      if (u < lo[k]) c = A[k] - lo[k];
      else if (u > hi[k]) c = A[k] - hi[k];
      else continue;
      num += c * D[k];
      den += D[k] * D[k];
    }
    if (den > 0.0) {
      double t = -num / den;
      if (t > ta && t < tb) {
        double e = seg_point_dist2(A, D, t, lo, hi);
        if (e < best) best = e;
      }
    }
  }
  return best;
}

/* Labels for N configurations (q is N x n). boxes: nbox rows of (lo[3], hi[3]).
 * label[j] = +1 in collision, -1 free. clearance[j] (optional) = min over links
 * and boxes of (distance - r), in metres.                                   */
void oracle_capsule_box_labels(int n, const double* dh, const double* base, int64_t N, const double* q,
                               double radius, int nbox, const double* boxes, int* label, double* clearance) {
#pragma omp parallel for schedule(dynamic, 256)
  for (int64_t j = 0; j < N; ++j) {
    double T[16 * 65];
    oracle_frames(n, dh, base, q + (size_t)n * j, T);
    double best = INFINITY;
    for (int i = 1; i <= n; ++i) {
      const double A[3] = {T[16 * (i - 1) + 3], T[16 * (i - 1) + 7], T[16 * (i - 1) + 11]};
      const double B[3] = {T[16 * i + 3], T[16 * i + 7], T[16 * i + 11]};
      for (int b = 0; b < nbox; ++b) {
        double d2 = oracle_segment_box_dist2(A, B, boxes + 6 * b, boxes + 6 * b + 3);
        double dist = sqrt(d2);
        if (dist - radius < best) best = dist - radius;
      }
    }
    label[j] = (best <= 0.0) ? 1 : -1;
    if (clearance) clearance[j] = best;
  }
}

/* Threads the oracle's OpenMP loops use (1 without OpenMP). */
int oracle_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* Sets the thread count of later OpenMP loops (no effect without OpenMP). */
void oracle_set_num_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}
