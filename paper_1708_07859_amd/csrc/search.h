// Searches of sorted 32-bit keys with short chains of dependent loads.
//
// A bisection over n keys is log2(n) loads, each waiting for the one
// before.  A quinary step probes four positions spread over the candidate
// range with independent loads, issued together, and keeps the fifth of
// the range they bracket: about log5(n) dependent loads.  Used where one
// thread searches alone (a unit's probed key range), so the extra loads
// cost no occupancy.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lh {

// Number of entries <= x in the non-decreasing a[0, n), n < 2^32 - 1.
__device__ __forceinline__ uint32_t count_le_quinary(const uint32_t* a, uint32_t n, uint32_t x) {
  uint32_t L = 0, W = n + 1;  // the count lies in [L, L + W)
  while (W > 1) {
    uint32_t j[4], pv[4];
#pragma unroll
    for (int i = 0; i < 4; i++) {
      // probe positions in [L, L + W - 2]: an answer above position p
      // means a[p] <= x
      const uint32_t o = (uint32_t)(((uint64_t)(i + 1) * W) / 5u);
      const uint32_t oi = o ? o - 1 : 0u;
      j[i] = L + (oi < W - 2 ? oi : W - 2);
      pv[i] = a[j[i]];
    }
    uint32_t m = 0;
#pragma unroll
    for (int i = 0; i < 4; i++) m += pv[i] <= x ? 1u : 0u;
    // m probes hold keys <= x: the count is above probe m - 1 and at most
    // probe m (the probes are in increasing positions, so the m true ones
    // come first)
    uint32_t nl = L, nr = j[0];
#pragma unroll
    for (int i = 0; i < 4; i++)
      if (m == (uint32_t)i + 1) {
        nl = j[i] + 1;
        nr = i < 3 ? j[i < 3 ? i + 1 : 3] : L + W - 1;
      }
    L = nl;
    W = nr - nl + 1;
  }
  return L;
}

// First position in the sorted keys [b, e) holding a key >= x (e if none),
// through the level's line samples (samp[j] = keys[j * 32]): the samples of
// the lines starting inside [b, e) locate the line, then the line (or the
// range's partial first line) gives the position.
__device__ __forceinline__ uint32_t lower_bound_sampled_quinary(const uint32_t* keys, const uint32_t* samp, uint32_t b,
                                                                uint32_t e, uint32_t x) {
  if (b >= e || x == 0) return b;
  const uint32_t y = x - 1;  // keys < x are the keys <= y
  const uint32_t jf = (b + 31u) >> 5, jl = (e - 1) >> 5;
  const uint32_t k = jl >= jf ? count_le_quinary(samp + jf, jl - jf + 1, y) : 0u;
  const uint32_t sb = k ? (jf + k - 1) << 5 : b;
  const uint64_t se64 = (uint64_t)(jf + k) << 5;
  const uint32_t se = se64 < e ? (uint32_t)se64 : e;
  return sb + count_le_quinary(keys + sb, se - sb, y);
}

}  // namespace lh
