// Opt-in per-kernel-class timing with HIP events recorded on the launch
// stream.  When enabled, the transform launchers bracket each launch with an
// event pair; completed pairs are folded into per-class totals when the
// entry point finishes (its stream is synchronised by then).
#include "cs_internal.h"

#include <atomic>
#include <cstring>
#include <mutex>
#include <vector>

namespace csr {

namespace {
struct Pending {
  int cls;
  double bytes;
  hipEvent_t a, b;
};
struct Stat {
  int64_t launches = 0;
  double ms = 0.0;
  double bytes = 0.0;
};
std::atomic<int> g_on{0};
std::mutex g_mu;
std::vector<hipEvent_t> g_free;
std::vector<Pending> g_pending;
Stat g_stats[PC_COUNT];
const char* g_names[PC_COUNT] = {"col_fwd", "col_inv", "row_happly", "row_resid", "row_fwd", "row_adj"};

hipEvent_t get_event() {
  if (!g_free.empty()) {
    hipEvent_t e = g_free.back();
    g_free.pop_back();
    return e;
  }
  // Timing only: without the system-scope fence a recorded event does not
  // write back and invalidate the caches around the launch it brackets, so
  // the measured launch runs as it does without events.
  hipEvent_t e;
  CS_HIP(hipEventCreateWithFlags(&e, hipEventDisableSystemFence));
  return e;
}
}  // namespace

bool prof_on() { return g_on.load(std::memory_order_relaxed) != 0 && !no_alloc_mode(); }

int prof_begin(hipStream_t s, hipEvent_t* ev) {
  std::lock_guard<std::mutex> lk(g_mu);
  *ev = get_event();
  CS_HIP(hipEventRecord(*ev, s));
  return 0;
}

int prof_end(int cls, double bytes, hipEvent_t start, hipStream_t s) {
  std::lock_guard<std::mutex> lk(g_mu);
  hipEvent_t e = get_event();
  CS_HIP(hipEventRecord(e, s));
  g_pending.push_back({cls, bytes, start, e});
  return (int)g_pending.size() - 1;
}

void prof_discard(int idx) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (idx >= 0 && idx < (int)g_pending.size()) g_pending[idx].cls = -1;
}

void prof_flush() {
  std::lock_guard<std::mutex> lk(g_mu);
  for (auto& p : g_pending) {
    CS_HIP(hipEventSynchronize(p.b));
    float ms = 0.f;
    CS_HIP(hipEventElapsedTime(&ms, p.a, p.b));
    g_free.push_back(p.a);
    g_free.push_back(p.b);
    if (p.cls < 0) continue;   // a launch that found its work already done
    g_stats[p.cls].launches += 1;
    g_stats[p.cls].ms += ms;
    g_stats[p.cls].bytes += p.bytes;
  }
  g_pending.clear();
}

}  // namespace csr

using namespace csr;

extern "C" {

int cs_prof_enable(int on) { return g_on.exchange(on ? 1 : 0); }

void cs_prof_reset(void) {
  std::lock_guard<std::mutex> lk(g_mu);
  for (auto& s : g_stats) s = Stat{};
}

int cs_prof_read(cs_prof_stat* out, int max) {
  if (!out) return PC_COUNT;
  prof_flush();
  std::lock_guard<std::mutex> lk(g_mu);
  int n = 0;
  for (int c = 0; c < PC_COUNT && n < max; ++c) {
    std::memset(&out[n], 0, sizeof(cs_prof_stat));
    std::strncpy(out[n].name, g_names[c], sizeof(out[n].name) - 1);
    out[n].launches = g_stats[c].launches;
    out[n].total_ms = g_stats[c].ms;
    out[n].bytes = g_stats[c].bytes;
    ++n;
  }
  return n;
}

}  // extern "C"
