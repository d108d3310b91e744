// Opt-in per-phase timing with HIP events recorded on the launch stream, and
// a query of the per-merge sizes of the last solve.  Both exist for
// measurement (rooflines of individual kernels); neither is on by default.
#include <mutex>
#include <vector>

#include "phdc_internal.h"
#include "profile.h"

namespace phdc {

namespace {
struct Rec {
  int phase;
  hipEvent_t a, b;
};
std::mutex g_pm;
bool g_on = false;
uint32_t g_mask = 0xffffffffu;  // phases recorded while enabled
std::vector<Rec> g_recs;
std::vector<hipEvent_t> g_pool;

hipEvent_t take_event() {
  if (!g_pool.empty()) {
    hipEvent_t e = g_pool.back();
    g_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  hipEventCreate(&e);
  return e;
}
}  // namespace

ProfScope::ProfScope(int phase, hipStream_t s) : phase_(phase), s_(s), a_(nullptr) {
  std::lock_guard<std::mutex> lk(g_pm);
  if (!g_on || phase < 0 || phase >= 32 || !((g_mask >> phase) & 1u)) return;
  a_ = take_event();
  hipEventRecord((hipEvent_t)a_, s_);
}

ProfScope::~ProfScope() {
  if (!a_) return;
  std::lock_guard<std::mutex> lk(g_pm);
  hipEvent_t b = take_event();
  hipEventRecord(b, s_);
  g_recs.push_back(Rec{phase_, (hipEvent_t)a_, b});
}

}  // namespace phdc

using namespace phdc;

extern "C" {

int phdc_profile_enable(int on) {
  std::lock_guard<std::mutex> lk(g_pm);
  g_on = on != 0;
  return 0;
}

int phdc_profile_select(uint32_t mask) {
  std::lock_guard<std::mutex> lk(g_pm);
  g_mask = mask;
  return 0;
}

int phdc_profile_read(double* ms, int64_t* count, int nphase) {
  if (!ms || !count || nphase <= 0) return -1;
  std::lock_guard<std::mutex> lk(g_pm);
  for (int i = 0; i < nphase; ++i) {
    ms[i] = 0.0;
    count[i] = 0;
  }
  for (auto& r : g_recs) {
    hipEventSynchronize(r.b);
    float t = 0.f;
    hipEventElapsedTime(&t, r.a, r.b);
    if (r.phase >= 0 && r.phase < nphase) {
      ms[r.phase] += t;
      count[r.phase] += 1;
    }
    g_pool.push_back(r.a);
    g_pool.push_back(r.b);
  }
  g_recs.clear();
  return 0;
}

}  // extern "C"
