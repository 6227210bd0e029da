// A join that allocates no device memory, for callers that cannot allocate
// (tight serving loops, harnesses that forbid allocation).
//
// Every temporary of the join comes from one static device array per GPU,
// `scratch`, through the allocator's bump arena; the result is copied into
// buffers the caller owns.  The array's device address is taken once per
// device with hipGetSymbolAddress and only that address is used from the
// host: the array's name in host code is a host-side stand-in, not device
// memory.  All calls on one GPU share its array, so calls that overlap on
// one GPU race; every call leaves the array holding its own temporaries,
// and the join clears whatever it needs zeroed before using it.
#include <cstring>
#include <memory>
#include <mutex>

#include "engine.h"

static __device__ __align__(256) unsigned char scratch[LH_NOALLOC_SCRATCH_BYTES];

namespace lh {

namespace {

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[MAX_DEVICES] = {};

// The current device's copy of `scratch` (its address taken on first use).
void* scratch_for_current_device() {
  int dev = 0;
  LH_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= MAX_DEVICES) fail(LH_ERR_UNSUPPORTED, "noalloc: device id beyond the scratch table");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      (void)hipGetLastError();
      fail(LH_ERR_DEVICE, std::string("noalloc: hipGetSymbolAddress(scratch) failed: ") + hipGetErrorString(e));
    }
    register_arena_range(p, LH_NOALLOC_SCRATCH_BYTES);
    g_scratch_ptr[dev] = p;
  }
  return g_scratch_ptr[dev];
}

}  // namespace

uint64_t run_plan_noalloc(const lh_plan_t* p, hipStream_t s, uint64_t max_rows, uint32_t* const* out_keys,
                          uint64_t* counts, double* sums, uint64_t* peak_bytes) {
  if (p->blas) fail(LH_ERR_UNSUPPORTED, "noalloc: a BLAS plan (LH_DENSE_BLAS) allocates inside rocBLAS");
  Arena arena;
  arena.base = scratch_for_current_device();
  arena.cap = LH_NOALLOC_SCRATCH_BYTES;
  uint64_t n = 0;
  try {
    ArenaScope scope(arena);
    std::unique_ptr<lh_result_impl> res(run_plan(p, s));
    const lh_result& R = res->pub;
    n = R.n_rows;
    if (n > max_rows) {
      std::string msg = "noalloc: the result has " + std::to_string(n) + " rows, the output buffers hold " +
                        std::to_string(max_rows);
      fail(LH_ERR_OVERFLOW, msg);
    }
    if (n) {
      for (uint32_t c = 0; c < R.n_cols; c++)
        LH_HIP(hipMemcpyAsync(out_keys[c], R.out_keys[c], n * sizeof(uint32_t), hipMemcpyDeviceToDevice, s));
      LH_HIP(hipMemcpyAsync(counts, R.counts, n * sizeof(uint64_t), hipMemcpyDeviceToDevice, s));
      if (R.sums) LH_HIP(hipMemcpyAsync(sums, R.sums, n * sizeof(double), hipMemcpyDeviceToDevice, s));
    }
    LH_HIP(hipStreamSynchronize(s));
  } catch (...) {
    // work already queued may still use the scratch: let it finish before
    // the next call can hand the same memory out again
    (void)hipStreamSynchronize(s);
    (void)hipGetLastError();
    throw;
  }
  if (peak_bytes) *peak_bytes = arena.peak;
  return n;
}

}  // namespace lh
