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
// The launch shape -- queries per work item (16, 32 or 64), waves per
// workgroup (4 or 8), whether a wave interleaves the MFMAs of two query
// blocks, and the share of the resident capacity the persistent grid takes
// (all or three quarters) -- is chosen by timing the candidates on the actual
// batch (fastron_batch_autotune) and remembered per (moving points, support
// size bucket, precision, device) for later batches of the same kind. A round
// of queries can be captured once into a HIP graph (counter reset by a kernel,
// then the scoring launch) and replayed.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
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

template <int MM, typename R, int QB, bool RAT, bool PAIRED, int W>
__global__ void __launch_bounds__(64 * W) k_score_batched(ChainArgs c, const float* __restrict__ q,
                                                           const BatchItem* __restrict__ items, int64_t n_items,
                                                           unsigned long long* __restrict__ counter,
                                                           const float* __restrict__ tiles,
                                                           const int64_t* __restrict__ tile_off,
                                                           const float* __restrict__ f_const, int Mp, float gamma,
                                                           float* __restrict__ f, int8_t* __restrict__ label) {
  __shared__ f4 lds[W][64][MM];
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
    wave_score_fp32<MM, QB, RAT, PAIRED>(lds[wave], tiles + t0 * tile_floats(Mp), nt, Mp, f_const[it.env], it.q0,
                                         qend, f, label);
  }
}

// Launch shape of the batched kernel.
struct BatchShape {
  int qb = 4;        // query blocks of 16 per work item
  int waves = 4;     // waves per workgroup (4 or 8)
  int paired = 0;    // interleave two query blocks' MFMAs (qb >= 2)
  int occ_pct = 100; // share of the resident capacity the persistent grid takes (75 or 100)
};

template <int MM, typename R, bool RAT, int W>
static const void* batched_kernel_w(int qb, int paired) {
  if (qb == 1) return reinterpret_cast<const void*>(k_score_batched<MM, R, 1, RAT, false, W>);
  if (qb == 2)
    return paired ? reinterpret_cast<const void*>(k_score_batched<MM, R, 2, RAT, true, W>)
                  : reinterpret_cast<const void*>(k_score_batched<MM, R, 2, RAT, false, W>);
  return paired ? reinterpret_cast<const void*>(k_score_batched<MM, R, 4, RAT, true, W>)
                : reinterpret_cast<const void*>(k_score_batched<MM, R, 4, RAT, false, W>);
}

template <int MM, typename R>
static const void* batched_kernel_r(const BatchShape& sh, bool rat) {
  if (sh.waves == 8)
    return rat ? batched_kernel_w<MM, R, true, 8>(sh.qb, sh.paired) : batched_kernel_w<MM, R, false, 8>(sh.qb, sh.paired);
  return rat ? batched_kernel_w<MM, R, true, 4>(sh.qb, sh.paired) : batched_kernel_w<MM, R, false, 4>(sh.qb, sh.paired);
}

template <typename R>
static const void* batched_kernel_m(int mm, const BatchShape& sh, bool rat) {
#define FASTRON_BMM(K) \
  case K: return batched_kernel_r<K, R>(sh, rat);
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
  BatchShape shape;
  int shape_from_cache = 0;
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

// Tuned shapes, per (moving points, support-size bucket, precision, device
// architecture and CU count).
typedef std::tuple<int, int, int, std::string, int> ShapeKey;
std::mutex g_shape_mu;
std::map<ShapeKey, BatchShape>& shape_cache() {
  static std::map<ShapeKey, BatchShape> m;
  return m;
}

fastron_status shape_key(const fastron_batch* b, ShapeKey* key) {
  hipDeviceProp_t prop;
  FASTRON_HIP(hipGetDeviceProperties(&prop, b->device));
  // support bucket: log2 of the mean support-set size per environment
  const double mean_s = b->E > 0 ? (double)b->S_total / b->E : 0.0;
  const int bucket = mean_s >= 1.0 ? (int)std::floor(std::log2(mean_s)) : 0;
  *key = ShapeKey(b->c.Mm, bucket, (int)FASTRON_SCORE_FP32, std::string(prop.gcnArchName), prop.multiProcessorCount);
  return FASTRON_OK;
}

// Work items for the shape's query blocks, longest first.
fastron_status build_items(fastron_batch* b, const BatchShape& shape, hipStream_t s) {
  drop_graph(b);
  const int per = 16 * shape.qb;
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
  b->shape = shape;
  return FASTRON_OK;
}

fastron_status launch_batch(fastron_batch* b, const float* q, float* f, int8_t* label, hipStream_t s) {
  const ChainArgs& c = b->c;
  hipLaunchKernelGGL(k_reset_counter, dim3(1), dim3(64), 0, s, b->d_counter);
  FASTRON_HIP(hipGetLastError());
  if (b->n_items == 0) return FASTRON_OK;
  const bool rat = rational_sum_ok(c, b->gamma);
  const BatchShape& sh = b->shape;
  const void* kfn = c.n >= kFp64Joints ? batched_kernel_m<double>(c.Mm, sh, rat)
                                       : batched_kernel_m<float>(c.Mm, sh, rat);
  if (!kfn) return fail(FASTRON_EUNSUPPORTED, "batched scoring needs 1..16 moving control points");
  const int threads = 64 * sh.waves;
  int ncu = 0, per_cu = 0;
  FASTRON_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, b->device));
  FASTRON_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kfn, threads, 0));
  if (per_cu < 1) per_cu = 1;
  int64_t blocks = ((int64_t)ncu * per_cu * sh.occ_pct + 99) / 100;
  if (blocks < 1) blocks = 1;
  const int64_t need = (b->n_items + sh.waves - 1) / sh.waves;
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
  FASTRON_HIP(hipLaunchKernel(kfn, dim3((unsigned)blocks), dim3((unsigned)threads), args, 0, s));
  return FASTRON_OK;
}

bool valid_shape(const BatchShape& sh) {
  return (sh.qb == 1 || sh.qb == 2 || sh.qb == 4) && (sh.waves == 4 || sh.waves == 8) &&
         (sh.paired == 0 || (sh.paired == 1 && sh.qb >= 2)) && (sh.occ_pct == 75 || sh.occ_pct == 100);
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
  st = build_items(b, BatchShape(), nullptr);
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
  ShapeKey key;
  fastron_status st = shape_key(b, &key);
  if (st != FASTRON_OK) return st;
  if (tune_get("batch.shape_cache") == 1) {
    BatchShape cached;
    bool hit = false;
    {
      std::lock_guard<std::mutex> lk(g_shape_mu);
      auto it = shape_cache().find(key);
      if (it != shape_cache().end()) {
        cached = it->second;
        hit = true;
      }
    }
    if (hit) {
      b->shape_from_cache = 1;
      return build_items(b, cached, s);
    }
  }
  hipEvent_t e0, e1;
  FASTRON_HIP(hipEventCreate(&e0));
  FASTRON_HIP(hipEventCreate(&e1));
  BatchShape best;
  float best_ms = 1e30f;
  const int qbs[] = {1, 2, 4};
  for (int qb : qbs)
    for (int waves : {4, 8})
      for (int paired = 0; paired <= (qb >= 2 ? 1 : 0); ++paired)
        for (int occ : {100, 75}) {
          if (st != FASTRON_OK) break;
          BatchShape sh;
          sh.qb = qb;
          sh.waves = waves;
          sh.paired = paired;
          sh.occ_pct = occ;
          st = build_items(b, sh, s);
          if (st != FASTRON_OK) break;
          st = launch_batch(b, q, f, label, s);  // warm-up
          if (st != FASTRON_OK) break;
          hipError_t e = hipEventRecord(e0, s);
          for (int r = 0; r < 2 && st == FASTRON_OK && e == hipSuccess; ++r) st = launch_batch(b, q, f, label, s);
          if (e == hipSuccess) e = hipEventRecord(e1, s);
          if (e == hipSuccess) e = hipEventSynchronize(e1);
          float ms = 0.f;
          if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
          if (e != hipSuccess && st == FASTRON_OK) st = fail(FASTRON_EHIP, "autotune timing failed: %s", hipGetErrorString(e));
          if (st == FASTRON_OK && ms < best_ms) {
            best_ms = ms;
            best = sh;
          }
        }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st != FASTRON_OK) return st;
  {
    std::lock_guard<std::mutex> lk(g_shape_mu);
    shape_cache()[key] = best;
  }
  b->shape_from_cache = 0;
  return build_items(b, best, s);
}

fastron_status fastron_batch_get_shape(const fastron_batch* b, int32_t* queries_per_item, int32_t* waves_per_group,
                                       int32_t* paired, int32_t* grid_pct, int32_t* from_cache) {
  clear_error();
  FASTRON_CHECK(b != nullptr, "batch is NULL");
  if (queries_per_item) *queries_per_item = 16 * b->shape.qb;
  if (waves_per_group) *waves_per_group = b->shape.waves;
  if (paired) *paired = b->shape.paired;
  if (grid_pct) *grid_pct = b->shape.occ_pct;
  if (from_cache) *from_cache = b->shape_from_cache;
  return FASTRON_OK;
}

fastron_status fastron_batch_set_shape(fastron_batch* b, int32_t queries_per_item, int32_t waves_per_group,
                                       int32_t paired, int32_t grid_pct, void* stream) {
  clear_error();
  FASTRON_CHECK(b != nullptr, "batch is NULL");
  BatchShape sh;
  sh.qb = queries_per_item / 16;
  sh.waves = waves_per_group;
  sh.paired = paired;
  sh.occ_pct = grid_pct;
  FASTRON_CHECK(queries_per_item % 16 == 0 && valid_shape(sh),
                "shape (%d queries, %d waves, paired %d, grid %d%%) is not one of the tuned candidates",
                queries_per_item, waves_per_group, paired, grid_pct);
  b->shape_from_cache = 0;
  return build_items(b, sh, as_stream(stream));
}

int32_t fastron_batch_tile_queries(const fastron_batch* b) { return b ? 16 * b->shape.qb : -1; }

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
