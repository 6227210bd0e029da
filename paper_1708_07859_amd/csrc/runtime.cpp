// Error plumbing and stream-ordered device allocation.
#include <atomic>
#include <cstdlib>
#include <cstring>
#include <sstream>

#include "lh_internal.h"

namespace lh {

void fail(lh_status st, const std::string& msg) { throw Error{st, msg}; }

void hip_fail(hipError_t e, const char* what, const char* file, int line) {
  std::ostringstream os;
  os << what << " failed: " << hipGetErrorString(e) << " (" << file << ":" << line << ")";
  lh_status st = (e == hipErrorOutOfMemory) ? LH_ERR_OOM : LH_ERR_DEVICE;
  throw Error{st, os.str()};
}

namespace {
std::atomic<long> g_live{0};
std::atomic<long> g_allocs{0};
long g_fail_after = -2;  // -2: not read yet, -1: never

long fail_after() {
  if (g_fail_after == -2) {
    const char* e = std::getenv("LH_FAULT_ALLOC_AFTER");
    g_fail_after = e ? std::atol(e) : -1;
  }
  return g_fail_after;
}

bool g_pool_configured = false;

void configure_pool() {
  if (g_pool_configured) return;
  int dev = 0;
  LH_HIP(hipGetDevice(&dev));
  hipMemPool_t pool;
  if (hipDeviceGetDefaultMemPool(&pool, dev) == hipSuccess) {
    uint64_t thr = UINT64_MAX;  // keep freed blocks cached for reuse
    (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &thr);
  }
  g_pool_configured = true;
}
}  // namespace

void* dalloc(size_t bytes, hipStream_t s) {
  if (bytes == 0) return nullptr;
  configure_pool();
  long fa = fail_after();
  long k = g_allocs.fetch_add(1);
  if (fa >= 0 && k >= fa) fail(LH_ERR_OOM, "injected allocation failure (LH_FAULT_ALLOC_AFTER)");
  void* p = nullptr;
  hipError_t e = hipMallocAsync(&p, bytes, s);
  if (e != hipSuccess || !p) {
    (void)hipGetLastError();
    std::ostringstream os;
    os << "device allocation of " << bytes << " bytes failed: " << hipGetErrorString(e);
    fail(e == hipErrorOutOfMemory ? LH_ERR_OOM : LH_ERR_DEVICE, os.str());
  }
  g_live.fetch_add(1);
  return p;
}

void dfree(void* p, hipStream_t s) {
  if (!p) return;
  (void)hipFreeAsync(p, s);
  g_live.fetch_sub(1);
}

long live_allocations() { return g_live.load(); }

}  // namespace lh

// ---------------------------------------------------------------------------
// Opt-in kernel timing
// ---------------------------------------------------------------------------
#include <map>
#include <mutex>

namespace lh {

namespace {
struct Pending {
  std::string name;
  hipEvent_t e0, e1;
  uint64_t rows, elems;
};
struct Agg {
  uint64_t launches = 0, rows = 0, elems = 0;
  double ms = 0;
};
std::mutex g_prof_mu;
bool g_prof_on = false;
std::vector<Pending> g_pending;
std::map<std::string, Agg> g_agg;

void resolve_pending() {
  for (auto& p : g_pending) {
    float ms = 0;
    if (hipEventSynchronize(p.e1) == hipSuccess && hipEventElapsedTime(&ms, p.e0, p.e1) == hipSuccess) {
      Agg& a = g_agg[p.name];
      a.launches++;
      a.ms += ms;
      a.rows += p.rows;
      a.elems += p.elems;
    }
    (void)hipEventDestroy(p.e0);
    (void)hipEventDestroy(p.e1);
  }
  g_pending.clear();
}
}  // namespace

bool prof_enabled() { return g_prof_on; }

ProfScope::ProfScope(const char* n, hipStream_t st, uint64_t r, uint64_t el) : name(n), s(st), rows(r), elems(el) {
  if (!g_prof_on) return;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    e0 = e1 = nullptr;
    return;
  }
  (void)hipEventRecord(e0, s);
}

ProfScope::~ProfScope() {
  if (!e0) return;
  (void)hipEventRecord(e1, s);
  std::lock_guard<std::mutex> lk(g_prof_mu);
  g_pending.push_back(Pending{name, e0, e1, rows, elems});
}

}  // namespace lh

extern "C" {

void lh_profile_enable(int on) {
  std::lock_guard<std::mutex> lk(lh::g_prof_mu);
  lh::g_prof_on = on != 0;
}

void lh_profile_reset(void) {
  std::lock_guard<std::mutex> lk(lh::g_prof_mu);
  lh::resolve_pending();
  lh::g_agg.clear();
}

uint32_t lh_profile_read(lh_profile_entry* out, uint32_t max_entries) {
  std::lock_guard<std::mutex> lk(lh::g_prof_mu);
  lh::resolve_pending();
  uint32_t i = 0;
  for (auto& kv : lh::g_agg) {
    if (out && i < max_entries) {
      lh_profile_entry& e = out[i];
      memset(&e, 0, sizeof e);
      strncpy(e.name, kv.first.c_str(), sizeof(e.name) - 1);
      e.launches = kv.second.launches;
      e.total_ms = kv.second.ms;
      e.rows = kv.second.rows;
      e.elements = kv.second.elems;
    }
    i++;
  }
  return i;
}

}  // extern "C"
