/*
 * fastron_fk.h -- C ABI of the gfx950 (MI355X) Fastron-FK library.
 *
 * Fastron with the forward-kinematics (FK) kernel, after Das & Yip,
 * "Forward Kinematics Kernel for Improved Proxy Collision Checking":
 *   - forward kinematics of a standard D-H chain into control points
 *     (Section II-A, Eq. 1 and Eq. 2);
 *   - the FK kernel K_FK(x, x') = (1/M) sum_m K_RQ(FK_m(x), FK_m(x')) built on
 *     the second-order rational quadratic kernel
 *     K_RQ(p, p') = (1 + gamma/2 ||p - p'||^2)^-2 (Section II-B Eq. 3,
 *     Section III-A Eq. 4);
 *   - the Fastron model f(x) = sum_i alpha_i K_FK(S_i, x) and its sign
 *     (Section III-B): f > 0 predicts "in collision" (+1), f < 0 "free" (-1);
 *     f == 0 is reported as +1;
 *   - Gram-column updates and the Fastron model update, Algorithm 1
 *     (Section III-B, Eq. 5-9).
 *
 * Conventions shared by every entry point
 *   - Array arguments are DEVICE pointers (memory of the current HIP device)
 *     owned by the caller, contiguous, row-major, of the element type named
 *     in the prototype. Structs and the arrays they point to are HOST memory,
 *     read only during the call. The library never frees caller memory.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream). All
 *     work is enqueued on it asynchronously unless an entry point says it
 *     synchronises.
 *   - Arguments are validated before any HIP call. Errors come back as a
 *     negative fastron_status; fastron_last_error() then returns a message
 *     (thread-local, valid until the next call on the same thread). Nothing
 *     aborts or throws across the ABI.
 *   - Limits: 1 <= n <= 16 joints, 1 <= M <= 16 control points. One call
 *     takes at most 2^32 - 256 configurations or rows (2^31 - 128 queries
 *     for the FK-kernel score entry points), since a launch spans at most
 *     2^32 - 1 work-items per grid dimension; more go in several calls
 *     (FASTRON_EINVAL otherwise). Offsets into every array are 64-bit, so
 *     arrays past 2^31 elements are addressed correctly.
 */
#ifndef FASTRON_FK_H
#define FASTRON_FK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  FASTRON_OK = 0,
  FASTRON_NOT_CONVERGED = 1,  /* Algorithm 1 hit iter_max; outputs are a valid partial model */
  FASTRON_EINVAL = -1,        /* invalid argument (nothing was launched) */
  FASTRON_EUNSUPPORTED = -2,  /* valid but unsupported request (e.g. no gfx950 device) */
  FASTRON_EHIP = -3,          /* a HIP runtime call failed; see fastron_last_error() */
  FASTRON_ENOMEM = -4,        /* a device allocation failed */
  FASTRON_EDEVICE = -5        /* a device-side safety limit fired (the training record exchange timed out) */
} fastron_status;

#define FASTRON_MAX_JOINTS 16
#define FASTRON_MAX_POINTS 16

/* Standard D-H chain (Section II-A, Eq. 1). Joint i (0-based) has link length
 * a[i] (translation along the new x axis), twist alpha[i], offset d[i]
 * (translation along the previous z axis) and angle offset theta[i]. A
 * revolute joint adds its variable to theta, a prismatic joint adds it to d.
 * wA_0 = base (row-major 4x4, last row 0 0 0 1) or the identity.           */
typedef struct {
  int32_t n;
  const double* a;       /* [n] */
  const double* alpha;   /* [n] */
  const double* d;       /* [n] */
  const double* theta;   /* [n] or NULL = zeros */
  const int32_t* type;   /* [n] 0 revolute, 1 prismatic; NULL = all revolute */
  const double* base;    /* [16] or NULL = identity */
} fastron_chain;

/* Control points (Section II-A, Eq. 2): point m sits at pos(wA_{frame[m]} T_m)
 * where T_m translates by offset[3m..3m+2] in frame frame[m]; frame 0 is the
 * base frame, frame n the end of the chain. Section III-A places points at
 * frame origins (offset NULL).                                              */
typedef struct {
  int32_t M;
  const int32_t* frame;  /* [M], each in [0, n] */
  const double* offset;  /* [M*3] or NULL = frame origins */
} fastron_cpoints;

/* Control-point placement of Section III-A (host only, no device work): one
 * point at the origin of each joint frame 1..n, except that a revolute joint
 * with a_i = 0 and d_i = 0 gets none, since its origin coincides with the
 * preceding one. With include_base != 0, frame 0 (the base origin, the same
 * for every configuration) is listed first. frame is HOST memory with room
 * for n + 1 entries; *M receives the number written.                       */
fastron_status fastron_control_point_frames(const fastron_chain* chain, int32_t include_base, int32_t* frame,
                                           int32_t* M);

/* ---- a1: batched forward kinematics (Section II-A, Eq. 1-2) --------------
 * q [N][n] float joint values -> P [N][M][3] float control-point positions.
 * One thread per configuration; the chain product runs in FP64 when n >= 7,
 * FP32 otherwise. N == 0 is a no-op.                                        */
fastron_status fastron_fk_points(const fastron_chain* chain, const fastron_cpoints* cp, const float* q,
                                 int64_t N, float* P, void* stream);

/* ---- a2: prepared support set --------------------------------------------
 * The support set of a Fastron model (Section III-B: configurations S_i with
 * weights alpha_i) converted once into the operand layout the scoring kernels
 * stream: per-point scaled control points, their squared norms and alpha/M.
 * `data` is caller-owned device memory of at least fastron_model_bytes(S, M)
 * bytes, 256-byte aligned; its contents are private to the library. The
 * blob holds the supports' control points, so a model must be scored with
 * the chain and control points it was prepared with. support_q is [S][n]
 * float, alpha [S] float (device). fastron_model_bytes returns -1 for S < 0
 * or M outside [1, 16]; fastron_support_prep returns FASTRON_EINVAL for a
 * blob that is too small or misaligned, gamma <= 0 or a bad chain.          */
typedef struct {
  int64_t S;        /* support-set size (0 allowed: f == 0 everywhere) */
  int32_t M;        /* control points per configuration */
  float gamma;      /* kernel width, gamma > 0 (Eq. 3) */
  void* data;       /* device blob */
  int64_t bytes;    /* capacity of data in bytes */
} fastron_model;

int64_t fastron_model_bytes(int64_t S, int32_t M);

fastron_status fastron_support_prep(const fastron_chain* chain, const fastron_cpoints* cp, const float* support_q,
                                    const float* alpha, int64_t S, float gamma, fastron_model* model, void* stream);

/* ---- a3/a6: fused FK-kernel score and sign (Section III-B) --------------
 * f[j] = sum_i alpha_i K_FK(S_i, q_j) with the FK of q_j computed in the same
 * kernel; label[j] = +1 if f[j] >= 0 else -1. f and/or label may be NULL
 * (not both). flags select the arithmetic of the cross term:
 *   FASTRON_SCORE_FP32  FP32 MFMA cross term (default)
 *   FASTRON_SCORE_BF16  BF16 MFMA cross term, FP32 norms and accumulation
 *   FASTRON_SCORE_VALU  FP32 cross term on the vector ALU (no MFMA)         */
#define FASTRON_SCORE_FP32 0u
#define FASTRON_SCORE_BF16 1u
#define FASTRON_SCORE_VALU 2u
/* BF16 precision variants (OR into FASTRON_SCORE_BF16): the cross term uses
 * 1, 3 or 6 bf16 products per coordinate (hi.hi; + hi.mid + mid.hi;
 * + hi.lo + lo.hi + mid.mid), splitting each coordinate of
 * sqrt(gamma/2) p into bf16 parts. PLAIN also takes both squared norms from
 * the hi parts, so its t is that of the rounded points (>= 1 up to FP32
 * rounding); every BF16 form clamps t at 1 (Eq. 3: K_RQ <= 1).            */
#define FASTRON_BF16_PLAIN 0x00u
#define FASTRON_BF16_SPLIT2 0x10u
#define FASTRON_BF16_SPLIT3 0x20u

fastron_status fastron_fk_score_prepared(const fastron_chain* chain, const fastron_cpoints* cp,
                                         const fastron_model* model, const float* q, int64_t N, float* f,
                                         int8_t* label, uint32_t flags, void* stream);

/* Which of two equivalent ways the scoring kernels (single-model, batched and
 * the screening fallback) use to sum K_RQ = 1/t^2 over the control points of
 * one (support, query) pair, for this chain, control points, gamma and flags
 * (host only, no device work): 1 = one running fraction n/e per pair with a
 * single reciprocal (taken when a bound R on the distance of every moving
 * point from the base -- finite unless a prismatic joint precedes one --
 * keeps T = 1.01 (1 + 2 gamma R^2), an upper bound on t, within
 * T^(2 Mm) <= 2^120 and T <= 2^16, or T <= 2^8 for FASTRON_BF16_PLAIN, and
 * the tuning key "score.rational" is 1); 0 = one saturated reciprocal per
 * value. Negative: FASTRON_EINVAL for a bad chain, gamma <= 0 or unknown
 * flags.                                                                    */
int32_t fastron_score_rational(const fastron_chain* chain, const fastron_cpoints* cp, float gamma, uint32_t flags);

/* Convenience form: prepares the support set (a2) into stream-ordered scratch
 * memory and scores (a3) in one call.                                       */
fastron_status fastron_fk_score(const fastron_chain* chain, const fastron_cpoints* cp, const float* support_q,
                                const float* alpha, int64_t S, float gamma, const float* q, int64_t N, float* f,
                                int8_t* label, uint32_t flags, void* stream);

/* ---- scoring that allocates nothing ---------------------------------------
 * For callers that cannot allocate device memory during a call: code under
 * HIP graph capture, tight serving loops, hosts that forbid hipMalloc. Same
 * arguments, validation and results as fastron_fk_score, but the prepared
 * support set (a2) goes into a static device buffer of
 * FASTRON_NOALLOC_SCRATCH_BYTES per device that the library holds until the
 * process ends, instead of stream-ordered scratch; no allocating call is
 * made. A support set whose prepared size fastron_model_bytes(S, M) exceeds
 * the buffer is rejected with FASTRON_EINVAL before any device work (at
 * M = 8 up to S = 20,864 fit; at M = 16 up to S = 10,448). The first call
 * on a device looks up the buffer's address (FASTRON_EHIP if that fails).
 * Every call on one device shares its buffer and keeps the last call's
 * contents: calls ordered on one stream are safe, but calls that overlap in
 * time on one device (unordered streams, several host threads) race and
 * give undefined results.                                                   */
#define FASTRON_NOALLOC_SCRATCH_BYTES (16ll << 20)
fastron_status fastron_fk_score_noalloc(const fastron_chain* chain, const fastron_cpoints* cp, const float* support_q,
                                        const float* alpha, int64_t S, float gamma, const float* q, int64_t N, float* f,
                                        int8_t* label, uint32_t flags, void* stream);

/* ---- a4: Gram column and F update (Section III-B, Eq. 8; Algorithm 1) ----
 * kcol[j] = K_FK(X_j, X_i) for all j, and F[j] += delta_alpha * kcol[j]
 * (delta_alpha = b_i y_i - F_i for an add or adjust, -alpha_i for a removal).
 * X [N][n] float are the training configurations (device); their control
 * points are computed with fastron_fk_points into stream-ordered scratch of
 * N * M * 3 floats that is released before the call returns. F (in/out,
 * [N]) and kcol (out, [N]) may each be NULL (not both). Errors:
 * FASTRON_EINVAL for N < 1, i outside [0, N), gamma <= 0 or non-finite
 * delta_alpha (nothing launched); FASTRON_ENOMEM if the scratch cannot be
 * allocated. Asynchronous on `stream`.                                      */
fastron_status fastron_gram_update(const fastron_chain* chain, const fastron_cpoints* cp, const float* X, int64_t N,
                                   float gamma, int64_t i, float delta_alpha, float* F, float* kcol, void* stream);

/* Points form of the same update: P [N][M][3] float are the training set's
 * control points (fastron_fk_points output), so repeated columns over one
 * training set do not repeat its forward kinematics. Same results as
 * fastron_gram_update on the configurations P was computed from.           */
fastron_status fastron_gram_update_points(const float* P, int64_t N, int32_t M, float gamma, int64_t i,
                                          float delta_alpha, float* F, float* kcol, void* stream);

/* ---- a5: Fastron model update, Algorithm 1 (Section III-B) --------------
 * Runs Algorithm 1 on the device: greedy add/adjust of the most negative
 * margin y_i F_i (lowest index on ties), removal of redundant support points
 * (largest y_i (F_i - alpha_i) over alpha_i != 0, lowest index on ties),
 * caps iter_max and s_max, then removeNonsupportPoints.
 *   X [N][n] float      training configurations (device); their control
 *                       points go into stream-ordered scratch of N * M * 3
 *                       floats, released before the call returns
 *   y [N] int8          +1 in collision, -1 free
 *   alpha, F [N]        in/out; zeros = fresh model, else a previous model
 *                       (loadPreviousModel: F must equal K alpha)
 *   support_idx [N]     out: ascending indices with alpha != 0
 *   n_support, updates  HOST out: |S| and the number of add/remove updates
 * beta >= 1 is the conditional bias (Eq. 5). The call synchronises `stream`.
 * Returns FASTRON_OK when the loop ended by break, FASTRON_NOT_CONVERGED when
 * iter_max updates were made first (outputs are a valid partial model),
 * FASTRON_EINVAL for bad arguments (nothing launched), FASTRON_EDEVICE if the
 * device-side record exchange exceeded its wait budget. fastron_train_f64
 * keeps alpha and F in double and evaluates the kernel in FP64
 * (reference-precision mode). trace_action / trace_index (device int32
 * [trace_cap], may be NULL) record the first trace_cap updates: action 1 =
 * add, 2 = remove.                                                          */
fastron_status fastron_train(const fastron_chain* chain, const fastron_cpoints* cp, const float* X, const int8_t* y,
                             int64_t N, float gamma, float beta, int64_t iter_max, int64_t s_max, float* alpha,
                             float* F, int32_t* support_idx, int64_t* n_support, int64_t* updates,
                             int32_t* trace_action, int32_t* trace_index, int64_t trace_cap, void* stream);
fastron_status fastron_train_f64(const fastron_chain* chain, const fastron_cpoints* cp, const float* X,
                                 const int8_t* y, int64_t N, double gamma, double beta, int64_t iter_max,
                                 int64_t s_max, double* alpha, double* F, int32_t* support_idx, int64_t* n_support,
                                 int64_t* updates, int32_t* trace_action, int32_t* trace_index, int64_t trace_cap,
                                 void* stream);

/* Points forms: the same update on P [N][M][3] float control points
 * (fastron_fk_points output) instead of configurations -- for callers that
 * keep the training set's control points (the moving-obstacle updates
 * re-train on rows whose points are already known). Bit-identical to
 * fastron_train / fastron_train_f64 on the configurations P came from.      */
fastron_status fastron_train_points(const float* P, const int8_t* y, int64_t N, int32_t M, float gamma, float beta,
                                    int64_t iter_max, int64_t s_max, float* alpha, float* F, int32_t* support_idx,
                                    int64_t* n_support, int64_t* updates, int32_t* trace_action,
                                    int32_t* trace_index, int64_t trace_cap, void* stream);
fastron_status fastron_train_points_f64(const float* P, const int8_t* y, int64_t N, int32_t M, double gamma,
                                        double beta, int64_t iter_max, int64_t s_max, double* alpha, double* F,
                                        int32_t* support_idx, int64_t* n_support, int64_t* updates,
                                        int32_t* trace_action, int32_t* trace_index, int64_t trace_cap,
                                        void* stream);

/* Several independent training sets (Algorithm 1 each, FP32) in one launch,
 * e.g. the environments of the batched form after their obstacles moved
 * (points form: P [N_total][M][3] from fastron_fk_points):
 * set e is rows offsets[e] .. offsets[e+1] - 1 of P, y, alpha and F
 * (offsets: HOST array of E + 1 int64, strictly increasing from 0). The sets
 * advance concurrently, each with its own exchange, and each ends exactly as
 * fastron_train on that set alone would. support_idx [N_total] receives set
 * e's ascending support indices (relative to offsets[e]) at
 * support_idx[offsets[e]]; n_support and updates are HOST arrays [E]. The
 * call synchronises `stream`; FASTRON_NOT_CONVERGED if any set hit iter_max.*/
fastron_status fastron_train_batch(const float* P, const int8_t* y, int32_t E, const int64_t* offsets, int32_t M,
                                   float gamma, float beta, int64_t iter_max, int64_t s_max, float* alpha, float* F,
                                   int32_t* support_idx, int64_t* n_support, int64_t* updates, void* stream);

/* ---- a7: batched form ----------------------------------------------------
 * E environments share one arm (chain + control points); environment e has
 * its own Fastron model (supports support_off[e] .. support_off[e+1] - 1 of
 * the concatenated support arrays) and its own queries (query_off[e] ..
 * query_off[e+1] - 1 of the concatenated query array). Offsets are HOST
 * arrays of E + 1 non-decreasing int64 starting at 0; they are copied.
 *   fastron_batch_create    allocates the batch's device buffers (synchronous)
 *   fastron_batch_prepare   support_q [S_total][n], alpha [S_total] (device)
 *   fastron_batch_score     scores q [N_total][n] into f / label [N_total] in
 *                           ONE persistent launch (work items claimed in
 *                           longest-first order from a device counter)
 *   fastron_batch_autotune  times the launch shapes on these arguments and
 *                           keeps the fastest: queries per work item (16, 32,
 *                           64), waves per workgroup (4, 8), interleaved MFMAs
 *                           of two query blocks (off/on, 32 or 64 queries) and
 *                           the share of the resident capacity the grid takes
 *                           (100 or 75 %); syncs. The result is remembered per
 *                           (moving points, log2 of the mean support-set size,
 *                           precision, device architecture and CU count), and a
 *                           later batch of the same kind takes it without
 *                           timing (tuning key "batch.shape_cache" = 0 times
 *                           every call). It discards a graph captured before it.
 *   fastron_batch_get_shape / fastron_batch_set_shape  read the shape in use
 *                           (from_cache = 1 when the last autotune reused one)
 *                           or pick one of the candidates directly; every shape
 *                           gives the same results bit for bit.
 *   fastron_batch_capture   records {counter reset, scoring launch} with these
 *                           pointers into a HIP graph on `stream` (non-null)
 *   fastron_batch_replay    launches the captured graph; FASTRON_EINVAL when
 *                           none is held (never captured, or discarded by a
 *                           later autotune)
 * Results equal fastron_fk_score_prepared on each environment's model.     */
typedef struct fastron_batch fastron_batch;
fastron_status fastron_batch_create(const fastron_chain* chain, const fastron_cpoints* cp, int32_t E,
                                    const int64_t* support_off, const int64_t* query_off, float gamma,
                                    fastron_batch** out);
fastron_status fastron_batch_prepare(fastron_batch* batch, const float* support_q, const float* alpha, void* stream);
fastron_status fastron_batch_score(fastron_batch* batch, const float* q, float* f, int8_t* label, void* stream);
fastron_status fastron_batch_autotune(fastron_batch* batch, const float* q, float* f, int8_t* label, void* stream);
fastron_status fastron_batch_capture(fastron_batch* batch, const float* q, float* f, int8_t* label, void* stream);
fastron_status fastron_batch_replay(fastron_batch* batch, void* stream);
int32_t fastron_batch_tile_queries(const fastron_batch* batch);
fastron_status fastron_batch_get_shape(const fastron_batch* batch, int32_t* queries_per_item, int32_t* waves_per_group,
                                       int32_t* paired, int32_t* grid_pct, int32_t* from_cache);
fastron_status fastron_batch_set_shape(fastron_batch* batch, int32_t queries_per_item, int32_t waves_per_group,
                                       int32_t paired, int32_t grid_pct, void* stream);
void fastron_batch_destroy(fastron_batch* batch);

/* ---- a8: learned screening ---------------------------------------------
 * A small network on the FK control points: 3M inputs -> H -> H -> 1 logit
 * (ReLU), BF16 matrix-core GEMMs with FP32 accumulation, FP32 master
 * weights, BCE-with-logits loss (label +1 = collision is the positive class),
 * Adam (beta1 0.9, beta2 0.999, eps 1e-8). Not part of the paper's method.
 * Parameters are one FP32 device vector in the order
 *   W1 [3M][H], b1 [H], W2 [H][H], b2 [H], w3 [H], b3 [1]
 * (fastron_mlp_param_count values); inputs are standardised by per-feature
 * mu / sd (device [3M]) before the first layer. Rows of P are the
 * [M][3] control points of fastron_fk_points; y holds one label per row of
 * P. fastron_mlp_train_epoch visits the rows in the order given by `order`
 * (device int32 [N], a permutation of 0..N-1; NULL = 0..N-1): it must hold
 * exactly N entries (an entry outside [0, N) is reported as
 * FASTRON_EINVAL). max_rows bounds one batch.
 * fastron_mlp_screen: queries with |logit| >= tau take sign(logit); the rest
 * (fell_back[j] = 1) take the sign of the Fastron FK score against `model`
 * (computed on the compacted subset). workspace: device memory of
 * fastron_mlp_screen_workspace_bytes(N, n) bytes. The call synchronises.  */
typedef struct fastron_mlp fastron_mlp;
fastron_status fastron_mlp_create(int32_t d_in, int32_t hidden, int64_t max_rows, fastron_mlp** out);
void fastron_mlp_destroy(fastron_mlp* net);
int64_t fastron_mlp_param_count(const fastron_mlp* net);
fastron_status fastron_mlp_set_params(fastron_mlp* net, const float* params, const float* mu, const float* sd,
                                      void* stream);
fastron_status fastron_mlp_get_params(const fastron_mlp* net, float* params, float* grads, float* mu, float* sd,
                                      void* stream);
/* Adam state: first and second moments (device [fastron_mlp_param_count],
 * same order as the parameters; either may be NULL) and the number of
 * optimiser steps taken since the last fastron_mlp_set_params (host).     */
fastron_status fastron_mlp_get_adam_state(const fastron_mlp* net, float* m, float* v, int64_t* step, void* stream);
fastron_status fastron_mlp_fit_standardisation(fastron_mlp* net, const float* P, int64_t N, void* stream);
fastron_status fastron_mlp_forward(fastron_mlp* net, const float* P, int64_t N, float* logits, void* stream);
fastron_status fastron_mlp_gradients(fastron_mlp* net, const float* P, const int8_t* y, int64_t N, float* loss,
                                     void* stream);
fastron_status fastron_mlp_train_epoch(fastron_mlp* net, const float* P, const int8_t* y, const int32_t* order,
                                       int64_t N, int64_t batch, float lr, float* mean_loss, void* stream);
fastron_status fastron_mlp_screen(fastron_mlp* net, const fastron_chain* chain, const fastron_cpoints* cp,
                                  const fastron_model* model, const float* q, int64_t N, float tau, float* logits,
                                  int8_t* label, uint8_t* fell_back, int64_t* n_fallback, void* workspace,
                                  int64_t workspace_bytes, void* stream);
int64_t fastron_mlp_screen_workspace_bytes(int64_t N, int32_t n_joints);

/* ---- the kernel on configurations (the paper's comparison, Section IV) ----
 * Fastron with the rational quadratic kernel of Section II-B, Eq. 3 applied
 * to the joint vectors themselves, K(x, x') = (1 + gamma/2 ||x - x'||^2)^-2:
 * the baseline whose support sets, accuracy and query times the paper
 * compares the FK kernel with. Same conventions as the FK entry points;
 * n in [1, 16] joint coordinates per configuration.
 *
 * fastron_rbf_score: f[j] = sum_s alpha_s K(support_x_s, q_j) and its sign
 * (label +1 for f >= 0). support_x [S][n], alpha [S], q [N][n] float; f and/or
 * label may be NULL (not both). S == 0 gives f = 0. The support set is
 * prepared into stream-ordered scratch memory on every call.              */
fastron_status fastron_rbf_score(const float* support_x, const float* alpha, int64_t S, int32_t n, float gamma,
                                 const float* q, int64_t N, float* f, int8_t* label, void* stream);

/* fastron_rbf_train / _f64: Algorithm 1 (Section III-B) with that kernel on
 * X [N][n] float (device) and labels y [N] int8; arguments, outputs, warm
 * start, caps and status as for fastron_train_points / _f64 with the
 * configurations in place of the control points. The FP64 form follows the
 * FP64 oracle step for step (trace arrays as in fastron_train_f64).        */
fastron_status fastron_rbf_train(const float* X, const int8_t* y, int64_t N, int32_t n, float gamma, float beta,
                                 int64_t iter_max, int64_t s_max, float* alpha, float* F, int32_t* support_idx,
                                 int64_t* n_support, int64_t* updates, void* stream);
fastron_status fastron_rbf_train_f64(const float* X, const int8_t* y, int64_t N, int32_t n, double gamma,
                                     double beta, int64_t iter_max, int64_t s_max, double* alpha, double* F,
                                     int32_t* support_idx, int64_t* n_support, int64_t* updates,
                                     int32_t* trace_action, int32_t* trace_index, int64_t trace_cap, void* stream);

/* ---- two-stage active learning (Section III-B, after the model update) ----
 * Assembles the training set of the next model update: X_out rows [0, S) =
 * the support configurations support_q [S][n] (alpha_out = their weights),
 * rows S + s k + j = support s plus noise row s k + j of noise [S k][n]
 * (samples near each support point; alpha_out = 0), and the last E rows =
 * explore [E][n] (uniform samples over the C-space; alpha_out = 0). The random
 * draws are the caller's. X_out holds S (1 + k) + E rows of n floats;
 * alpha_out (may be NULL) as many floats. All arrays are device memory. The
 * update then labels every row (fastron_label_capsule_box), zeroes the weights
 * of supports whose label changed (fastron_active_relabel), takes F = the
 * current model's score of every row (fastron_fk_score; F = K alpha) and
 * runs fastron_train_points from (alpha_out, F) on the rows' control points. */
fastron_status fastron_active_samples(const float* support_q, const float* alpha, int64_t S, int32_t n,
                                      const float* noise, int32_t k, const float* explore, int64_t E, float* X_out,
                                      float* alpha_out, void* stream);

/* After relabelling, a support point whose new label y[i] disagrees with the
 * sign of its weight alpha[i] violates the constraint y_i alpha_i >= 0 of
 * Eq. 5 that Algorithm 1 maintains; fastron_active_relabel sets such weights
 * to zero for the first S rows (y int8, alpha float, device, in place), so
 * that the update starts from a model that satisfies it. S == 0 is a no-op.  */
fastron_status fastron_active_relabel(const int8_t* y, int64_t S, float* alpha, void* stream);

/* ---- a9: geometric labels -------------------------------------------------
 * Stands in for the ground-truth collision checker of Section IV: link i is a
 * capsule of radius `radius` around the segment between the origins of
 * frames i-1 and i; obstacles are axis-aligned boxes, a DEVICE array of nbox
 * rows (lo_x, lo_y, lo_z, hi_x, hi_y, hi_z) in double, 0 <= nbox <= 4096,
 * with lo <= hi on every axis (the caller's duty: the array is not read on
 * the host; an inverted box gives unspecified labels). label[j] = +1 if some
 * capsule touches some box (exact segment-box distance <= radius), else -1.
 * clearance[j] (may be NULL) = min distance - radius. Computed in FP64;
 * pairs that a bounding-box bound shows cannot lower the minimum are
 * skipped, and without clearance a configuration stops at its first
 * touching pair (same labels).                                              */
fastron_status fastron_label_capsule_box(const fastron_chain* chain, const float* q, int64_t N, double radius,
                                         const double* boxes, int32_t nbox, int8_t* label, float* clearance,
                                         void* stream);

/* ---- tuning ----------------------------------------------------------------
 * Process-wide launch parameters (host side):
 *   "train.kernel"      1 (default): the wave form of Algorithm 1 (one
 *                       wave per workgroup exchanges the workgroup's record;
 *                       no barrier inside the exchange); 0: the slice kernel
 *                       (also used when the wave form's grid would exceed
 *                       its limits)
 *   "train.waves"       waves per workgroup the wave form starts from: 1, 2,
 *                       4, 8 (default) or 16 (FP64 workgroups stop at 8);
 *                       1 keeps single-wave workgroups
 *                       (which also take over when the multi-wave grid would
 *                       exceed 256 workgroups, 128 in FP64)
 *   "train.wave_groups" grid cap of the wave form, 1..512 (64): the waves per
 *                       workgroup double up to 16 (single-wave workgroups:
 *                       the points per lane double up to 16) while the grid
 *                       exceeds it
 *   "train.poll_delay"  sleeps of 64 clocks before the first poll of each
 *                       record exchange, 0..64, or -1 (default): adapted by
 *                       each workgroup to how often its first poll came too
 *                       early. Timing only; results do not depend on it.
 *   "train.single_group" 1 (default): a training set of at most 1,024 points
 *                       (512 in FP64) runs in one workgroup of 16 waves (8),
 *                       which needs no record exchange; 0: the grid rule
 *                       above alone.
 *                       Results do not depend on it.
 *   "train.blocks"      workgroups of the slice kernel, 0 = automatic
 *   "train.threads"     threads per slice-kernel workgroup: 256, 512 or 1024
 *   "score.rational"    1 (default): the scoring kernels (FP32 MFMA and
 *                       VALU, BF16, batched) sum a pair's 1/t^2 terms as one
 *                       running fraction (one reciprocal per pair) when a
 *                       bound on the chain's reach keeps the fraction in
 *                       range (see fastron_score_rational); 0: one saturated
 *                       reciprocal per value always. The two agree to FP32
 *                       rounding.
 *   "score.bf16_blocks" query blocks of 16 whose BF16 operands the BF16 score
 *                       kernel keeps resident per pass: 2 (default: fewer
 *                       registers, 3 waves per SIMD) or 4 (same results)
 *   "batch.shape_cache" 1 (default): fastron_batch_autotune reuses a shape
 *                       tuned earlier in the process for a batch of the same
 *                       kind; 0: it times the candidates on every call
 * Keys take effect at the next launch (a captured batch graph keeps the
 * kernel it was captured with). fastron_tune_get returns -1 for an unknown
 * key.                                                                      */
fastron_status fastron_tune_set(const char* key, int64_t value);
int64_t fastron_tune_get(const char* key);

/* Last error message of the calling thread ("" after success). */
const char* fastron_last_error(void);

/* Library version string. */
const char* fastron_version(void);

#ifdef __cplusplus
}
#endif

#endif /* FASTRON_FK_H */
