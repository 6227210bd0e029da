// Wave64 / block primitives for gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lh {

constexpr int WAVE = 64;

__device__ __forceinline__ int lane_id() { return __lane_id(); }

// Workgroups are dispatched to the 8 XCDs (each with its own L2) in turn:
// block b runs on XCD b % 8.  This renumbers blocks so that each XCD owns
// one contiguous range of logical block ids (when the grid is a multiple of
// 8), keeping neighbouring work, which reads neighbouring data, on one L2.
constexpr uint32_t N_XCD = 8;
__device__ __forceinline__ uint32_t xcd_block(uint32_t b, uint32_t grid) {
  if (grid % N_XCD) return b;
  return (b % N_XCD) * (grid / N_XCD) + b / N_XCD;
}

// A run of n keys at p, cut into 16-byte chunks on the 16-byte grid: chunk
// c holds the run's elements 4c - head .. 4c - head + 3 (those in [0, n)).
struct KeyRun {
  const uint32_t* al;   // p rounded down to 16 bytes
  uint32_t head, n, nch;
};

__device__ __forceinline__ KeyRun key_run(const uint32_t* p, uint32_t n) {
  KeyRun r;
  r.head = (uint32_t)(((uintptr_t)p & 15u) >> 2);
  r.al = p - r.head;
  r.n = n;
  r.nch = n ? (r.head + n + 3) / 4 : 0u;
  return r;
}

// Chunk c of a run: one 16-byte load when the chunk lies inside the run,
// else its elements inside the run one by one (the rest are 0).
__device__ __forceinline__ uint4 load_chunk(const KeyRun& r, uint32_t c) {
  const int64_t e0 = 4 * (int64_t)c - r.head;
  if (e0 >= 0 && e0 + 4 <= (int64_t)r.n) return *reinterpret_cast<const uint4*>(r.al + 4 * (uint64_t)c);
  uint32_t v[4];
#pragma unroll
  for (int k = 0; k < 4; k++) {
    const int64_t e = e0 + k;
    v[k] = (e >= 0 && e < (int64_t)r.n) ? r.al[4 * (uint64_t)c + k] : 0u;
  }
  return make_uint4(v[0], v[1], v[2], v[3]);
}

__device__ __forceinline__ uint32_t chunk_elem(const uint4& x, int k) {
  return k == 0 ? x.x : k == 1 ? x.y : k == 2 ? x.z : x.w;
}

// Number of set bits of `mask` in lanes below this lane (mbcnt).
__device__ __forceinline__ uint32_t lanes_below(uint64_t mask) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                   __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }

template <class T>
__device__ __forceinline__ T wave_incl_scan(T v) {
  const int lane = lane_id();
#pragma unroll
  for (int d = 1; d < WAVE; d <<= 1) {
    T u = __shfl_up(v, d, WAVE);
    if (lane >= d) v += u;
  }
  return v;
}

template <class T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int d = WAVE / 2; d > 0; d >>= 1) v += __shfl_xor(v, d, WAVE);
  return v;
}

// Exclusive scan across a block of NT threads; `lds` holds NT/64 entries.
// Returns this thread's exclusive prefix and writes the block total.
template <class T, int NT>
__device__ __forceinline__ T block_excl_scan(T v, T* lds, T& total) {
  constexpr int NW = NT / WAVE;
  const int w = threadIdx.x / WAVE;
  T inc = wave_incl_scan(v);
  if (lane_id() == WAVE - 1) lds[w] = inc;
  __syncthreads();
  T off = 0, tot = 0;
#pragma unroll
  for (int i = 0; i < NW; i++) {
    T x = lds[i];
    if (i < w) off += x;
    tot += x;
  }
  __syncthreads();
  total = tot;
  return off + inc - v;
}

template <class T, int NT>
__device__ __forceinline__ T block_sum(T v, T* lds) {
  T total;
  (void)block_excl_scan<T, NT>(v, lds, total);
  return total;
}

// Largest index i in [lo, hi) with a[i] <= x, given a non-decreasing array
// whose a[lo] <= x (a load-balanced-search helper).
template <class T>
__device__ __forceinline__ uint64_t upper_bound_minus1(const T* a, uint64_t lo, uint64_t hi, T x) {
  // invariant: a[lo] <= x, answer in [lo, hi)
  while (hi - lo > 1) {
    uint64_t mid = lo + (hi - lo) / 2;
    if (a[mid] <= x) lo = mid; else hi = mid;
  }
  return lo;
}

// First index in [lo, hi) whose value is >= x (hi if none).
__device__ __forceinline__ uint32_t lower_bound_u32(const uint32_t* a, uint32_t lo, uint32_t hi, uint32_t x) {
  while (lo < hi) {
    uint32_t mid = lo + (hi - lo) / 2;
    if (a[mid] < x) lo = mid + 1; else hi = mid;
  }
  return lo;
}

}  // namespace lh
