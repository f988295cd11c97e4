// Batched form: many environments' Fastron models (same arm, uneven support
// sets and query batches) scored in one persistent launch.
//
// Work items are (environment, block of 16 * QB queries). Their cost is
// proportional to the environment's support-set size times the queries in
// the block, so the host sorts them by decreasing cost once (longest
// processing time first) and the device claims them in that order from an
// atomic counter: every wave loops, takes the next item, stages its queries'
// FK in LDS and streams that environment's support tiles (the same FP32 MFMA
// wave loop as the single-model kernel). The grid is sized to the resident
// capacity of the device, so waves never wait for a dispatch slot, and the
// loop ends for every wave once the counter passes the last item.
//
// The tile shape (QB) is chosen by timing the candidates on the actual batch
// (fastron_batch_autotune). A round of queries can be captured once into a
// HIP graph (counter reset by a kernel, then the scoring launch) and replayed.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "score_device.h"

struct fastron_batch;

namespace fastron {

struct BatchItem {
  int32_t env;
  int32_t nq;
  int64_t q0;
};

__global__ void k_reset_counter(unsigned long long* counter) {
  if (threadIdx.x == 0) *counter = 0ull;
}

template <int MM, typename R, int QB, bool RAT>
__global__ void __launch_bounds__(256) k_score_batched(ChainArgs c, const float* __restrict__ q,
                                                        const BatchItem* __restrict__ items, int64_t n_items,
                                                        unsigned long long* __restrict__ counter,
                                                        const float* __restrict__ tiles,
                                                        const int64_t* __restrict__ tile_off,
                                                        const float* __restrict__ f_const, int Mp, float gamma,
                                                        float* __restrict__ f, int8_t* __restrict__ label) {
  __shared__ f4 lds[kWavesPerBlock][64][MM];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (;;) {
    unsigned long long idx = 0ull;
    if (lane == 0) idx = atomicAdd(counter, 1ull);
    idx = __shfl(idx, 0);
    if (idx >= (unsigned long long)n_items) break;
    const BatchItem it = items[idx];
    const int64_t qend = it.q0 + it.nq;
    // the previous item's LDS reads of this wave are complete before it is overwritten
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    stage_queries<MM, R>(c, q, qend, gamma, it.q0 + lane, lds[wave]);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const int64_t t0 = tile_off[it.env];
    const int64_t nt = tile_off[it.env + 1] - t0;
    wave_score_fp32<MM, QB, RAT, false>(lds[wave], tiles + t0 * tile_floats(Mp), nt, Mp, f_const[it.env], it.q0, qend, f,
                            label);
  }
}

template <int MM, typename R, bool RAT>
static const void* batched_kernel_q(int qb) {
  switch (qb) {
    case 1: return reinterpret_cast<const void*>(k_score_batched<MM, R, 1, RAT>);
    case 2: return reinterpret_cast<const void*>(k_score_batched<MM, R, 2, RAT>);
    default: return reinterpret_cast<const void*>(k_score_batched<MM, R, 4, RAT>);
  }
}

template <int MM, typename R>
static const void* batched_kernel_r(int qb, bool rat) {
  return rat ? batched_kernel_q<MM, R, true>(qb) : batched_kernel_q<MM, R, false>(qb);
}

template <typename R>
static const void* batched_kernel_m(int mm, int qb, bool rat) {
#define FASTRON_BMM(K) \
  case K: return batched_kernel_r<K, R>(qb, rat);
  switch (mm) {
    FASTRON_BMM(1) FASTRON_BMM(2) FASTRON_BMM(3) FASTRON_BMM(4) FASTRON_BMM(5) FASTRON_BMM(6) FASTRON_BMM(7)
    FASTRON_BMM(8) FASTRON_BMM(9) FASTRON_BMM(10) FASTRON_BMM(11) FASTRON_BMM(12) FASTRON_BMM(13)
    FASTRON_BMM(14) FASTRON_BMM(15) FASTRON_BMM(16)
    default: return nullptr;
  }
#undef FASTRON_BMM
}

}  // namespace fastron

using namespace fastron;

struct fastron_batch {
  ChainArgs c;
  int E = 0;
  float gamma = 0.f;
  int Mp = 4;
  int qb = 4;
  int device = 0;
  int64_t S_total = 0, N_total = 0, total_tiles = 0;
  std::vector<int64_t> support_off, query_off, tile_off;
  int64_t* d_support_off = nullptr;
  int64_t* d_tile_off = nullptr;
  float* d_tiles = nullptr;
  float* d_fconst = nullptr;
  BatchItem* d_items = nullptr;
  int64_t n_items = 0;
  int64_t items_cap = 0;
  unsigned long long* d_counter = nullptr;
  bool prepared = false;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

namespace {

void drop_graph(fastron_batch* b);

void free_batch(fastron_batch* b) {
  if (!b) return;
  drop_graph(b);
  (void)hipFree(b->d_support_off);
  (void)hipFree(b->d_tile_off);
  (void)hipFree(b->d_tiles);
  (void)hipFree(b->d_fconst);
  (void)hipFree(b->d_items);
  (void)hipFree(b->d_counter);
  delete b;
}

// A captured graph holds the launch it recorded by value (kernel, grid and
// item count), so it does not follow a rebuilt work list: drop it, and let a
// replay report that it has to be captured again.
void drop_graph(fastron_batch* b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->exec = nullptr;
  b->graph = nullptr;
}

// Work items for tile shape qb, longest first.
fastron_status build_items(fastron_batch* b, int qb, hipStream_t s) {
  drop_graph(b);
  const int per = 16 * qb;
  std::vector<BatchItem> items;
  for (int e = 0; e < b->E; ++e) {
    const int64_t q0 = b->query_off[e], q1 = b->query_off[e + 1];
    for (int64_t j = q0; j < q1; j += per) items.push_back({e, (int32_t)std::min<int64_t>(per, q1 - j), j});
  }
  std::stable_sort(items.begin(), items.end(), [&](const BatchItem& x, const BatchItem& y) {
    const int64_t cx = (b->tile_off[x.env + 1] - b->tile_off[x.env]) * (int64_t)x.nq;
    const int64_t cy = (b->tile_off[y.env + 1] - b->tile_off[y.env]) * (int64_t)y.nq;
    return cx > cy;
  });
  b->n_items = (int64_t)items.size();
  if (b->n_items > b->items_cap) return fail(FASTRON_EINVAL, "internal: item list larger than its buffer");
  if (b->n_items > 0)
    FASTRON_HIP(hipMemcpyAsync(b->d_items, items.data(), items.size() * sizeof(BatchItem), hipMemcpyHostToDevice, s));
  FASTRON_HIP(hipStreamSynchronize(s));  // the host vector dies at return
  b->qb = qb;
  return FASTRON_OK;
}

fastron_status launch_batch(fastron_batch* b, const float* q, float* f, int8_t* label, hipStream_t s) {
  const ChainArgs& c = b->c;
  hipLaunchKernelGGL(k_reset_counter, dim3(1), dim3(64), 0, s, b->d_counter);
  FASTRON_HIP(hipGetLastError());
  if (b->n_items == 0) return FASTRON_OK;
  const bool rat = rational_sum_ok(c, b->gamma);
  const void* kfn = c.n >= kFp64Joints ? batched_kernel_m<double>(c.Mm, b->qb, rat)
                                       : batched_kernel_m<float>(c.Mm, b->qb, rat);
  if (!kfn) return fail(FASTRON_EUNSUPPORTED, "batched scoring needs 1..16 moving control points");
  int ncu = 0, per_cu = 0;
  FASTRON_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, b->device));
  FASTRON_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kfn, 256, 0));
  if (per_cu < 1) per_cu = 1;
  int64_t blocks = (int64_t)ncu * per_cu;
  const int64_t need = (b->n_items + kWavesPerBlock - 1) / kWavesPerBlock;
  if (blocks > need) blocks = need;
  int Mp = b->Mp;
  float gamma = b->gamma;
  int64_t n_items = b->n_items;
  const float* tiles = b->d_tiles;
  const int64_t* tile_off = b->d_tile_off;
  const float* fconst = b->d_fconst;
  const BatchItem* items = b->d_items;
  unsigned long long* counter = b->d_counter;
  void* args[] = {const_cast<ChainArgs*>(&c), &q, &items, &n_items, &counter, &tiles, &tile_off, &fconst, &Mp,
                  &gamma, &f, &label};
  FASTRON_HIP(hipLaunchKernel(kfn, dim3((unsigned)blocks), dim3(256), args, 0, s));
  return FASTRON_OK;
}

}  // namespace

extern "C" {

fastron_status fastron_batch_create(const fastron_chain* chain, const fastron_cpoints* cp, int32_t E,
                                    const int64_t* support_off, const int64_t* query_off, float gamma,
                                    fastron_batch** out) {
  clear_error();
  FASTRON_CHECK(out != nullptr, "out is NULL");
  *out = nullptr;
  ChainArgs c;
  fastron_status st = pack_chain(chain, cp, &c, true);
  if (st != FASTRON_OK) return st;
  FASTRON_CHECK(E >= 1, "E = %d < 1", E);
  FASTRON_CHECK(support_off && query_off, "support_off and query_off must be non-NULL host arrays");
  FASTRON_CHECK(support_off[0] == 0 && query_off[0] == 0, "offsets must start at 0");
  for (int e = 0; e < E; ++e) {
    FASTRON_CHECK(support_off[e + 1] >= support_off[e], "support_off decreases at %d", e);
    FASTRON_CHECK(query_off[e + 1] >= query_off[e], "query_off decreases at %d", e);
  }
  FASTRON_CHECK(std::isfinite(gamma) && gamma > 0.f, "gamma must be finite and > 0");
  FASTRON_CHECK(c.Mm >= 1, "batched scoring needs at least one moving control point");
  fastron_batch* b = new fastron_batch();
  b->c = c;
  b->E = E;
  b->gamma = gamma;
  b->Mp = mp_of(c.M);
  b->support_off.assign(support_off, support_off + E + 1);
  b->query_off.assign(query_off, query_off + E + 1);
  b->tile_off.resize(E + 1);
  b->tile_off[0] = 0;
  for (int e = 0; e < E; ++e) b->tile_off[e + 1] = b->tile_off[e] + ntiles_of(support_off[e + 1] - support_off[e]);
  b->S_total = support_off[E];
  b->N_total = query_off[E];
  b->total_tiles = b->tile_off[E];
  int64_t cap = 0;
  for (int e = 0; e < E; ++e) cap += (query_off[e + 1] - query_off[e] + 15) / 16;
  b->items_cap = cap;
  hipError_t err = hipGetDevice(&b->device);
  auto alloc = [&](void** p, size_t bytes) {
    if (err == hipSuccess) err = hipMalloc(p, bytes > 0 ? bytes : 256);
  };
  alloc(reinterpret_cast<void**>(&b->d_support_off), sizeof(int64_t) * (E + 1));
  alloc(reinterpret_cast<void**>(&b->d_tile_off), sizeof(int64_t) * (E + 1));
  alloc(reinterpret_cast<void**>(&b->d_tiles), (size_t)b->total_tiles * tile_floats(b->Mp) * sizeof(float));
  alloc(reinterpret_cast<void**>(&b->d_fconst), sizeof(float) * E);
  alloc(reinterpret_cast<void**>(&b->d_items), sizeof(BatchItem) * (size_t)cap);
  alloc(reinterpret_cast<void**>(&b->d_counter), 256);
  if (err == hipSuccess)
    err = hipMemcpy(b->d_support_off, support_off, sizeof(int64_t) * (E + 1), hipMemcpyHostToDevice);
  if (err == hipSuccess)
    err = hipMemcpy(b->d_tile_off, b->tile_off.data(), sizeof(int64_t) * (E + 1), hipMemcpyHostToDevice);
  if (err != hipSuccess) {
    free_batch(b);
    return fail(err == hipErrorOutOfMemory ? FASTRON_ENOMEM : FASTRON_EHIP, "batch allocation failed: %s",
                hipGetErrorString(err));
  }
  st = build_items(b, 4, nullptr);
  if (st != FASTRON_OK) {
    free_batch(b);
    return st;
  }
  *out = b;
  return FASTRON_OK;
}

fastron_status fastron_batch_prepare(fastron_batch* b, const float* support_q, const float* alpha, void* stream) {
  clear_error();
  FASTRON_CHECK(b != nullptr, "batch is NULL");
  FASTRON_CHECK(b->S_total == 0 || (support_q && alpha), "support_q and alpha must be non-NULL");
  fastron_status st = launch_prep_batched(b->c, support_q, alpha, b->d_support_off, b->d_tile_off, b->E,
                                          b->total_tiles, b->gamma, b->d_tiles, b->d_fconst, as_stream(stream));
  if (st == FASTRON_OK) b->prepared = true;
  return st;
}

fastron_status fastron_batch_score(fastron_batch* b, const float* q, float* f, int8_t* label, void* stream) {
  clear_error();
  FASTRON_CHECK(b != nullptr, "batch is NULL");
  FASTRON_CHECK(b->prepared, "fastron_batch_prepare has not been called");
  FASTRON_CHECK(b->N_total == 0 || q != nullptr, "q is NULL");
  FASTRON_CHECK(b->N_total == 0 || f != nullptr || label != nullptr, "f and label are both NULL");
  return launch_batch(b, q, f, label, as_stream(stream));
}

fastron_status fastron_batch_autotune(fastron_batch* b, const float* q, float* f, int8_t* label, void* stream) {
  clear_error();
  FASTRON_CHECK(b != nullptr, "batch is NULL");
  FASTRON_CHECK(b->prepared, "fastron_batch_prepare has not been called");
  FASTRON_CHECK(b->N_total == 0 || q != nullptr, "q is NULL");
  FASTRON_CHECK(b->N_total == 0 || f != nullptr || label != nullptr, "f and label are both NULL");
  hipStream_t s = as_stream(stream);
  hipEvent_t e0, e1;
  FASTRON_HIP(hipEventCreate(&e0));
  FASTRON_HIP(hipEventCreate(&e1));
  int best_qb = 4;
  float best = 1e30f;
  fastron_status st = FASTRON_OK;
  for (int qb : {1, 2, 4}) {
    st = build_items(b, qb, s);
    if (st != FASTRON_OK) break;
    st = launch_batch(b, q, f, label, s);  // warm-up
    if (st != FASTRON_OK) break;
    hipError_t e = hipEventRecord(e0, s);
    for (int r = 0; r < 3 && st == FASTRON_OK && e == hipSuccess; ++r) st = launch_batch(b, q, f, label, s);
    if (e == hipSuccess) e = hipEventRecord(e1, s);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e != hipSuccess) st = fail(FASTRON_EHIP, "autotune timing failed: %s", hipGetErrorString(e));
    if (st != FASTRON_OK) break;
    if (ms < best) {
      best = ms;
      best_qb = qb;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st != FASTRON_OK) return st;
  return build_items(b, best_qb, s);
}

int32_t fastron_batch_tile_queries(const fastron_batch* b) { return b ? 16 * b->qb : -1; }

fastron_status fastron_batch_capture(fastron_batch* b, const float* q, float* f, int8_t* label, void* stream) {
  clear_error();
  FASTRON_CHECK(b != nullptr, "batch is NULL");
  FASTRON_CHECK(b->prepared, "fastron_batch_prepare has not been called");
  FASTRON_CHECK(stream != nullptr, "capture needs a non-null stream");
  FASTRON_CHECK(b->N_total == 0 || q != nullptr, "q is NULL");
  FASTRON_CHECK(b->N_total == 0 || f != nullptr || label != nullptr, "f and label are both NULL");
  hipStream_t s = as_stream(stream);
  if (b->exec) {
    FASTRON_HIP(hipGraphExecDestroy(b->exec));
    b->exec = nullptr;
  }
  if (b->graph) {
    FASTRON_HIP(hipGraphDestroy(b->graph));
    b->graph = nullptr;
  }
  FASTRON_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
  fastron_status st = launch_batch(b, q, f, label, s);
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamEndCapture(s, &g);
  if (st != FASTRON_OK) {
    if (g) (void)hipGraphDestroy(g);
    return st;
  }
  if (e != hipSuccess) return fail(FASTRON_EHIP, "graph capture failed: %s", hipGetErrorString(e));
  b->graph = g;
  FASTRON_HIP(hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0));
  return FASTRON_OK;
}

fastron_status fastron_batch_replay(fastron_batch* b, void* stream) {
  clear_error();
  FASTRON_CHECK(b != nullptr && b->exec != nullptr,
                "no captured graph (call fastron_batch_capture first, and again after fastron_batch_autotune)");
  FASTRON_HIP(hipGraphLaunch(b->exec, as_stream(stream)));
  return FASTRON_OK;
}

void fastron_batch_destroy(fastron_batch* b) { free_batch(b); }

}  // extern "C"
