// Process-wide tuning table (host side). The autotuner and callers set launch
// parameters here; kernels never read it directly.
#include <cstring>
#include <mutex>
#include <string>
#include <unordered_map>

#include "fastron_internal.h"

namespace fastron {

namespace {
struct Knob {
  int64_t value;
  int64_t lo, hi;
  bool pow2;
};

std::mutex g_mu;
std::unordered_map<std::string, Knob>& table() {
  static std::unordered_map<std::string, Knob> t = {
      {"train.blocks", {0, 0, 4096, false}},    // 0 = automatic
      {"train.threads", {512, 256, 1024, true}},
      {"train.kernel", {1, 0, 1, false}},         // 1 = the wave form, 0 = the multi-wave slice kernel
      {"train.wave_groups", {64, 1, 512, false}},   // grid cap of the wave form
      {"train.waves", {8, 1, 16, true}},            // waves per workgroup of the wave form
      {"train.poll_delay", {-1, -1, 64, false}},    // sleeps before an exchange's first poll, -1 = adaptive
      {"train.single_group", {1, 0, 1, false}},     // 1: a set that fits one workgroup runs in one
      {"score.rational", {1, 0, 1, false}},        // 1 = running-fraction sum where the reach bound allows it
      {"score.bf16_blocks", {2, 2, 4, true}},      // query blocks resident per pass of the BF16 score kernel
      {"batch.shape_cache", {1, 0, 1, false}},     // 1 = batch autotune reuses a shape tuned for the same kind
  };
  return t;
}
}  // namespace

int64_t tune_get(const char* key) {
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = table().find(key);
  return it == table().end() ? -1 : it->second.value;
}

}  // namespace fastron

using namespace fastron;

extern "C" {

fastron_status fastron_tune_set(const char* key, int64_t value) {
  clear_error();
  FASTRON_CHECK(key != nullptr, "key is NULL");
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = table().find(key);
  FASTRON_CHECK(it != table().end(), "unknown tuning key '%s'", key);
  const Knob& k = it->second;
  FASTRON_CHECK(value >= k.lo && value <= k.hi, "%s = %lld outside [%lld, %lld]", key, (long long)value,
                (long long)k.lo, (long long)k.hi);
  FASTRON_CHECK(!k.pow2 || (value & (value - 1)) == 0, "%s must be a power of two", key);
  it->second.value = value;
  return FASTRON_OK;
}

int64_t fastron_tune_get(const char* key) {
  if (!key) return -1;
  return tune_get(key);
}

}  // extern "C"
