// Per-kernel timing with HIP events (measurement support).
#include <hip/hip_runtime.h>

#include <atomic>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "internal.hpp"
#include "launch.hpp"

namespace dgfs {
namespace prof {

struct Rec {
  std::string name;
  hipEvent_t a, b;
};
struct Stat {
  int64_t count = 0;
  double ms = 0.0;
};

static std::atomic<bool> g_on{false};
static std::mutex g_mu;
static std::vector<Rec> g_pending;
static std::vector<hipEvent_t> g_free;
static std::map<std::string, Stat> g_stats;

bool enabled() { return g_on.load(std::memory_order_relaxed); }

static hipEvent_t get_event() {
  if (!g_free.empty()) {
    hipEvent_t e = g_free.back();
    g_free.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  (void)hipEventCreate(&e);
  return e;
}

void *begin(const char *name, hipStream_t st) {
  std::lock_guard<std::mutex> lk(g_mu);
  Rec *r = new Rec{name, get_event(), get_event()};
  (void)hipEventRecord(r->a, st);
  return r;
}

void end(void *token, hipStream_t st) {
  Rec *r = static_cast<Rec *>(token);
  std::lock_guard<std::mutex> lk(g_mu);
  (void)hipEventRecord(r->b, st);
  g_pending.push_back(*r);
  delete r;
}

static void drain() {
  for (Rec &r : g_pending) {
    (void)hipEventSynchronize(r.b);
    float ms = 0.0f;
    if (hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
      Stat &s = g_stats[r.name];
      s.count += 1;
      s.ms += ms;
    }
    g_free.push_back(r.a);
    g_free.push_back(r.b);
  }
  g_pending.clear();
}

}  // namespace prof
}  // namespace dgfs

using namespace dgfs;

extern "C" dgfs_status dgfs_profile_enable(int32_t on) {
  std::lock_guard<std::mutex> lk(prof::g_mu);
  prof::drain();
  prof::g_stats.clear();
  prof::g_on.store(on != 0);
  return DGFS_OK;
}

extern "C" int32_t dgfs_profile_read(int32_t cap, char *names, int64_t *counts, double *total_ms) {
  std::lock_guard<std::mutex> lk(prof::g_mu);
  prof::drain();
  int32_t i = 0;
  for (auto &kv : prof::g_stats) {
    if (i < cap && names && counts && total_ms) {
      std::strncpy(names + 64 * i, kv.first.c_str(), 63);
      names[64 * i + 63] = 0;
      counts[i] = kv.second.count;
      total_ms[i] = kv.second.ms;
    }
    ++i;
  }
  return i;
}
