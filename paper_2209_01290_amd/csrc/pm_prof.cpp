// Kernel timing: while enabled, every launch the library makes is bracketed
// by two HIP events recorded on the launch's own stream; pm_prof_read()
// waits for them and sums the elapsed time per kernel name.
#include "pm_prof.hpp"

#include <atomic>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/pm.h"

namespace pm {
namespace {

struct Rec {
  const char* name;
  hipEvent_t a, b;
  bool closed;
};

std::atomic<int> g_on{0};
std::mutex g_mu;
std::vector<Rec> g_recs;
std::vector<hipEvent_t> g_free;
thread_local int g_off = 0;   // ProfOff nesting depth on this thread

hipEvent_t take_event() {
  if (!g_free.empty()) {
    hipEvent_t e = g_free.back();
    g_free.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

}  // namespace

ProfOff::ProfOff() { ++g_off; }
ProfOff::~ProfOff() { --g_off; }

ProfScope::ProfScope(hipStream_t s, const char* name) : s_(s), name_(name), slot_(-1) {
  if (g_off > 0 || !g_on.load(std::memory_order_relaxed)) return;
  std::lock_guard<std::mutex> lk(g_mu);
  Rec r{name, take_event(), take_event(), false};
  if (!r.a || !r.b) return;
  if (hipEventRecord(r.a, s) != hipSuccess) return;
  slot_ = (int)g_recs.size();
  g_recs.push_back(r);
}

void ProfScope::done() {
  if (slot_ < 0) return;
  std::lock_guard<std::mutex> lk(g_mu);
  Rec& r = g_recs[slot_];
  if (!r.closed && hipEventRecord(r.b, s_) == hipSuccess) r.closed = true;
  slot_ = -1;
}

}  // namespace pm

using namespace pm;

extern "C" int pm_prof_enable(int on) {
  g_on.store(on ? 1 : 0);
  return PM_OK;
}

extern "C" int pm_prof_read(pm_prof_entry* out, size_t cap, size_t* n_out, int reset) {
  std::lock_guard<std::mutex> lk(g_mu);
  std::map<std::string, pm_prof_entry> agg;
  int rc = PM_OK;
  for (Rec& r : g_recs) {
    if (!r.closed) continue;
    float ms = 0.f;
    if (hipEventSynchronize(r.b) != hipSuccess || hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess) {
      rc = PM_EHIP;
      continue;
    }
    pm_prof_entry& e = agg[r.name];
    if (e.launches == 0) {
      std::memset(e.name, 0, sizeof(e.name));
      std::strncpy(e.name, r.name, sizeof(e.name) - 1);
    }
    e.launches += 1;
    e.total_ms += ms;
  }
  size_t i = 0;
  for (auto& kv : agg) {
    if (out && i < cap) out[i] = kv.second;
    ++i;
  }
  if (n_out) *n_out = i;
  if (reset) {
    for (Rec& r : g_recs) {
      g_free.push_back(r.a);
      g_free.push_back(r.b);
    }
    g_recs.clear();
  }
  return rc;
}
