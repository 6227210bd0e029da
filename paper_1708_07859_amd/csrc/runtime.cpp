// Error plumbing and stream-ordered device allocation.
#include <atomic>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <sstream>
#include <unordered_map>
#include <vector>

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

// Freed blocks are kept and handed out again (a stream-ordered free and a
// fresh allocation each cost host time, milliseconds for large blocks).
// A cached block is reused only on the stream that freed it, so work still
// queued on that stream is ordered before the block's next use; every call
// of the library synchronizes its stream before it returns.  Sizes are
// rounded to 512 B below 1 MiB and to 2 MiB above; a block serves requests
// down to 4/5 of its size.  On an allocation failure the cache is released
// and the allocation retried.
namespace {
struct CachedBlock {
  void* p;
  hipStream_t s;
};
std::mutex g_cache_mu;
std::multimap<size_t, CachedBlock> g_free;      // cached blocks by capacity
std::unordered_map<void*, size_t> g_cap;        // capacity of every block held (live or cached)

size_t round_size(size_t b) {
  if (b <= (size_t(1) << 20)) return (b + 511) & ~size_t(511);
  const size_t g = size_t(2) << 20;
  return (b + g - 1) & ~(g - 1);
}

void release_cache(hipStream_t s) {
  std::lock_guard<std::mutex> lk(g_cache_mu);
  for (auto& kv : g_free) {
    (void)hipFreeAsync(kv.second.p, s);
    g_cap.erase(kv.second.p);
  }
  g_free.clear();
}
}  // namespace

// ---- bump arena -------------------------------------------------------------
// While an arena is active on a host thread, device allocations of that
// thread are carved from it in order and frees give nothing back until it
// ends; no device memory is allocated.  Memory inside a registered arena
// range is never handed to hipFreeAsync.
namespace {
thread_local Arena* t_arena = nullptr;
std::mutex g_arena_mu;
std::vector<std::pair<const char*, const char*>> g_arena_ranges;

bool in_arena_range(const void* p) {
  std::lock_guard<std::mutex> lk(g_arena_mu);
  const char* c = static_cast<const char*>(p);
  for (auto& r : g_arena_ranges)
    if (c >= r.first && c < r.second) return true;
  return false;
}
}  // namespace

void register_arena_range(void* base, size_t cap) {
  std::lock_guard<std::mutex> lk(g_arena_mu);
  const char* b = static_cast<const char*>(base);
  for (auto& r : g_arena_ranges)
    if (r.first == b) return;
  g_arena_ranges.emplace_back(b, b + cap);
}

bool arena_active() { return t_arena != nullptr; }

ArenaScope::ArenaScope(Arena& a) : prev(t_arena) {
  a.used = 0;
  t_arena = &a;
}
ArenaScope::~ArenaScope() { t_arena = prev; }

void* dalloc(size_t bytes, hipStream_t s) {
  if (bytes == 0) return nullptr;
  if (t_arena) {
    Arena& a = *t_arena;
    const size_t off = (a.used + 255) & ~size_t(255);
    if (off > a.cap || bytes > a.cap - off) {
      std::ostringstream os;
      os << "the static scratch of " << (a.cap >> 20) << " MiB cannot hold this join's temporaries (" << bytes
         << " more bytes at offset " << off << ")";
      fail(LH_ERR_OVERFLOW, os.str());
    }
    a.used = off + bytes;
    if (a.used > a.peak) a.peak = a.used;
    return static_cast<char*>(a.base) + off;
  }
  configure_pool();
  long fa = fail_after();
  long k = g_allocs.fetch_add(1);
  if (fa >= 0 && k >= fa) fail(LH_ERR_OOM, "injected allocation failure (LH_FAULT_ALLOC_AFTER)");
  const size_t want = round_size(bytes);
  {
    std::lock_guard<std::mutex> lk(g_cache_mu);
    for (auto it = g_free.lower_bound(want); it != g_free.end() && it->first <= want + want / 4; ++it) {
      if (it->second.s != s) continue;
      void* p = it->second.p;
      g_free.erase(it);
      g_live.fetch_add(1);
      return p;
    }
  }
  void* p = nullptr;
  hipError_t e = hipMallocAsync(&p, want, s);
  if (e == hipErrorOutOfMemory || (e == hipSuccess && !p)) {
    (void)hipGetLastError();
    release_cache(s);
    LH_HIP(hipStreamSynchronize(s));
    p = nullptr;
    e = hipMallocAsync(&p, want, s);
  }
  if (e != hipSuccess || !p) {
    (void)hipGetLastError();
    std::ostringstream os;
    os << "device allocation of " << bytes << " bytes failed: " << hipGetErrorString(e);
    fail(e == hipErrorOutOfMemory ? LH_ERR_OOM : LH_ERR_DEVICE, os.str());
  }
  {
    std::lock_guard<std::mutex> lk(g_cache_mu);
    g_cap[p] = want;
  }
  g_live.fetch_add(1);
  return p;
}

void dfree(void* p, hipStream_t s) {
  if (!p) return;
  if (in_arena_range(p)) return;   // arena memory is released when the arena ends
  std::lock_guard<std::mutex> lk(g_cache_mu);
  auto it = g_cap.find(p);
  if (it == g_cap.end()) {
    (void)hipFreeAsync(p, s);
  } else {
    g_free.emplace(it->second, CachedBlock{p, s});
  }
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
