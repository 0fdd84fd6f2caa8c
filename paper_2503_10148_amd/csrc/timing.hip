// Optional per-kernel timing with HIP events (sss_timing_* in sss.h).
#include <string.h>

#include <mutex>
#include <string>
#include <vector>

#include "common.hpp"

namespace sss {
namespace {

struct Pending {
  const char* name;
  hipEvent_t a, b;
};

struct Totals {
  std::string name;
  int64_t launches = 0;
  double ms = 0.0;
};

std::mutex g_mu;
bool g_on = false;
std::vector<Pending> g_pending;
std::vector<hipEvent_t> g_pool;
std::vector<Totals> g_totals;

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

// Resolve every pending pair (waits for it) into the totals; g_mu held.
void drain() {
  for (const Pending& p : g_pending) {
    float ms = 0.0f;
    if (hipEventSynchronize(p.b) == hipSuccess && hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
      Totals* t = nullptr;
      for (Totals& x : g_totals)
        if (x.name == p.name) t = &x;
      if (!t) {
        g_totals.push_back(Totals{p.name, 0, 0.0});
        t = &g_totals.back();
      }
      t->launches += 1;
      t->ms += ms;
    }
    g_pool.push_back(p.a);
    g_pool.push_back(p.b);
  }
  g_pending.clear();
}

}  // namespace

KernelTimer::KernelTimer(const char* name, hipStream_t st) : name_(name), st_(st) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_on) return;
  a_ = take_event();
  b_ = take_event();
  if (a_ && b_ && hipEventRecord(a_, st_) == hipSuccess) return;
  // no timing for this launch: hand the events back
  if (a_) g_pool.push_back(a_);
  if (b_) g_pool.push_back(b_);
  a_ = b_ = nullptr;
}

KernelTimer::~KernelTimer() {
  if (!a_ || !b_) return;
  std::lock_guard<std::mutex> lk(g_mu);
  if (hipEventRecord(b_, st_) == hipSuccess) {
    g_pending.push_back(Pending{name_, a_, b_});
  } else {
    g_pool.push_back(a_);
    g_pool.push_back(b_);
  }
}

}  // namespace sss

using namespace sss;

extern "C" {

int sss_timing_enable(int on) {
  std::lock_guard<std::mutex> lk(g_mu);
  g_on = on != 0;
  return SSS_OK;
}

void sss_timing_reset(void) {
  std::lock_guard<std::mutex> lk(g_mu);
  drain();
  g_totals.clear();
}

int sss_timing_read(sss_kernel_time_t* out, int max_entries) {
  if (!out || max_entries < 0) {
    set_error("sss_timing_read: null output or negative size");
    return SSS_ERR_INVALID;
  }
  std::lock_guard<std::mutex> lk(g_mu);
  drain();
  int k = 0;
  for (const Totals& t : g_totals) {
    if (k >= max_entries) break;
    memset(out[k].name, 0, sizeof(out[k].name));
    strncpy(out[k].name, t.name.c_str(), sizeof(out[k].name) - 1);
    out[k].launches = t.launches;
    out[k].total_ms = t.ms;
    ++k;
  }
  return k;
}

}  // extern "C"
