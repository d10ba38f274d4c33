// Process-wide launch profiler: a start/stop HIP event pair around each
// profiled launch, resolved and summed per kernel family at stop time.
#include <atomic>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "profile.h"

namespace fit {

namespace {
struct Rec {
  hipEvent_t a, b;
  const char* name;
};
std::mutex g_mu;
std::atomic<bool> g_on{false};
std::vector<Rec> g_recs;
std::vector<hipEvent_t> g_pool;

hipEvent_t take_event() {
  if (!g_pool.empty()) {
    hipEvent_t e = g_pool.back();
    g_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}
}  // namespace

int prof_begin(hipStream_t s) {
  if (!g_on.load(std::memory_order_relaxed)) return -1;
  std::lock_guard<std::mutex> lk(g_mu);
  hipEvent_t a = take_event(), b = take_event();
  if (!a || !b) return -1;
  if (hipEventRecord(a, s) != hipSuccess) return -1;
  g_recs.push_back(Rec{a, b, nullptr});
  return (int)g_recs.size() - 1;
}

void prof_end(int token, hipStream_t s, const char* name) {
  if (token < 0) return;
  std::lock_guard<std::mutex> lk(g_mu);
  if (token >= (int)g_recs.size()) return;
  g_recs[token].name = name;
  (void)hipEventRecord(g_recs[token].b, s);
}

}  // namespace fit

using namespace fit;

extern "C" fit_status fit_profile_start(void) {
  std::lock_guard<std::mutex> lk(g_mu);
  for (auto& r : g_recs) {
    g_pool.push_back(r.a);
    g_pool.push_back(r.b);
  }
  g_recs.clear();
  g_on.store(true);
  return FIT_OK;
}

extern "C" fit_status fit_profile_stop(fit_kernel_stat* out, int max, int* n) {
  g_on.store(false);
  std::lock_guard<std::mutex> lk(g_mu);
  std::map<std::string, std::pair<int64_t, double>> agg;
  fit_status st = FIT_OK;
  for (auto& r : g_recs) {
    if (!r.name) continue;
    if (hipEventSynchronize(r.b) != hipSuccess) {
      st = FIT_E_DEVICE;
      continue;
    }
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess) {
      st = FIT_E_DEVICE;
      continue;
    }
    auto& e = agg[r.name];
    e.first += 1;
    e.second += ms;
  }
  for (auto& r : g_recs) {
    g_pool.push_back(r.a);
    g_pool.push_back(r.b);
  }
  g_recs.clear();
  int k = 0;
  for (auto& kv : agg) {
    if (out && k < max) {
      std::memset(&out[k], 0, sizeof(fit_kernel_stat));
      std::strncpy(out[k].name, kv.first.c_str(), sizeof(out[k].name) - 1);
      out[k].launches = kv.second.first;
      out[k].total_ms = kv.second.second;
    }
    ++k;
  }
  if (n) *n = k;
  if (st != FIT_OK) set_error("fit_profile_stop: could not resolve some events");
  return st;
}
