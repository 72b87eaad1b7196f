// gmm_profile.hip -- optional per-kernel timing with HIP events.
//
// When enabled, the launchers record a pair of events on the caller's stream
// around every launch of the data-pass kernels (the ones that read all of X)
// and gmm_profile_read() accumulates their elapsed time per kernel kind.  It
// is meant for benchmarking eager calls; leave it disabled under graph
// capture.
#include <mutex>
#include <vector>

#include "gmm_internal.hpp"

namespace gmm {

namespace {

struct Rec {
  int kind;
  hipEvent_t a, b;
};

std::mutex g_mu;
bool g_on = false;
std::vector<Rec> g_pending;
double g_ms[kProfKinds];
int64_t g_n[kProfKinds];

}  // namespace

thread_local int tl_suppress = 0;

ProfSuppress::ProfSuppress() { ++tl_suppress; }
ProfSuppress::~ProfSuppress() { --tl_suppress; }

ProfScope::ProfScope(int kind, hipStream_t st) : kind_(kind), st_(st), a_(nullptr), b_(nullptr) {
  if (tl_suppress > 0) return;  // a caller that must not create events
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_on) return;
  if (hipEventCreate(&a_) != hipSuccess || hipEventCreate(&b_) != hipSuccess) {
    a_ = b_ = nullptr;
    return;
  }
  (void)hipEventRecord(a_, st_);
}

ProfScope::~ProfScope() {
  if (!a_) return;
  (void)hipEventRecord(b_, st_);
  std::lock_guard<std::mutex> lk(g_mu);
  g_pending.push_back({kind_, a_, b_});
}

static void drain_locked() {
  for (auto& r : g_pending) {
    float ms = 0.0f;
    if (hipEventSynchronize(r.b) == hipSuccess && hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess &&
        r.kind >= 0 && r.kind < kProfKinds) {
      g_ms[r.kind] += ms;
      g_n[r.kind] += 1;
    }
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  g_pending.clear();
}

}  // namespace gmm

extern "C" {

int gmm_profile_enable(int on) {
  std::lock_guard<std::mutex> lk(gmm::g_mu);
  gmm::drain_locked();
  for (int k = 0; k < gmm::kProfKinds; ++k) {
    gmm::g_ms[k] = 0.0;
    gmm::g_n[k] = 0;
  }
  gmm::g_on = on != 0;
  return GMM_OK;
}

int gmm_profile_read(int32_t kind, double* ms_total, int64_t* launches) {
  if (kind < 0 || kind >= gmm::kProfKinds || !ms_total || !launches) return GMM_EINVAL;
  std::lock_guard<std::mutex> lk(gmm::g_mu);
  gmm::drain_locked();
  *ms_total = gmm::g_ms[kind];
  *launches = gmm::g_n[kind];
  return GMM_OK;
}

}  // extern "C"
