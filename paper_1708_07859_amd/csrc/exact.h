// Exact, order-independent FP64 summation on the device.
//
// A sum of products is accumulated as a fixed-point integer whose least
// significant bit has weight 2^lsb, held in D signed 64-bit slots of 32-bit
// digits (slot i has weight 2^(lsb + 32 i)).  Contributions are added to the
// slots without carrying (each slot absorbs ~2^30 additions of 33-bit
// values), carries are propagated before slots are merged, and the final
// value is rounded once to the nearest double, ties to even.  Because
// integer addition is associative, the result does not depend on the order
// of the terms, the intersection algorithm, the set layout or the batching.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lh {

constexpr int EXACT_MAXD = 8;

// Exact product a*b = hi + lo (two-product via a fused multiply-add).
__device__ __forceinline__ void two_prod(double a, double b, double& hi, double& lo) {
  hi = __dmul_rn(a, b);
  lo = __fma_rn(a, b, -hi);
}

// Digits of |v| placed relative to 2^lsb: digit index k0 and three 32-bit
// (unnormalized, < 2^33) parts.  Returns false when v has bits below 2^lsb.
__device__ __forceinline__ bool split_to_digits(double v, int32_t lsb, int32_t& k0, int64_t& d0, int64_t& d1,
                                                int64_t& d2, bool& neg) {
  uint64_t bits = (uint64_t)__double_as_longlong(v);
  neg = (bits >> 63) != 0;
  uint32_t ex = (uint32_t)(bits >> 52) & 0x7ffu;
  uint64_t mant = bits & ((1ull << 52) - 1);
  int32_t e;
  if (ex == 0) {
    e = -1074;
  } else {
    mant |= 1ull << 52;
    e = (int32_t)ex - 1075;
  }
  if (mant == 0) {
    k0 = 0;
    d0 = d1 = d2 = 0;
    return true;
  }
  int32_t sh = e - lsb;
  if (sh < 0) {
    int tz = __builtin_ctzll(mant);
    if (tz < -sh) return false;
    mant >>= -sh;
    sh = 0;
  }
  k0 = sh >> 5;
  uint32_t off = (uint32_t)sh & 31u;
  uint64_t ml = mant & 0xffffffffull, mh = mant >> 32;
  uint64_t t0 = ml << off;   // < 2^64
  uint64_t t1 = mh << off;   // < 2^53
  d0 = (int64_t)(t0 & 0xffffffffull);
  d1 = (int64_t)((t0 >> 32) + (t1 & 0xffffffffull));
  d2 = (int64_t)(t1 >> 32);
  return true;
}

// Register accumulator with a compile-time slot count; D <= EXACT_MAXD
// slots are live.  Dynamic digit indices are resolved with selects so the
// slots stay in registers.
struct RegAcc {
  int64_t s[EXACT_MAXD];
  __device__ __forceinline__ void clear() {
#pragma unroll
    for (int i = 0; i < EXACT_MAXD; i++) s[i] = 0;
  }
  // Adds mult * v; returns false if v does not fit the window.
  __device__ __forceinline__ bool add(double v, int32_t lsb, uint32_t D, int64_t mult) {
    if (v == 0.0) return true;
    int32_t k0;
    int64_t d0, d1, d2;
    bool neg;
    if (!split_to_digits(v, lsb, k0, d0, d1, d2, neg)) return false;
    if (neg) mult = -mult;
    d0 *= mult;
    d1 *= mult;
    d2 *= mult;
    bool ok = (k0 < (int32_t)D) && (k0 + 1 < (int32_t)D || d1 == 0) && (k0 + 2 < (int32_t)D || d2 == 0);
#pragma unroll
    for (int i = 0; i < EXACT_MAXD; i++) {
      int64_t add = (i == k0) ? d0 : (i == k0 + 1) ? d1 : (i == k0 + 2) ? d2 : 0;
      s[i] += add;
    }
    return ok;
  }
  // Propagate carries so slots 0..D-2 hold digits in [0, 2^32).
  __device__ __forceinline__ void normalize(uint32_t D) {
    int64_t c = 0;
#pragma unroll
    for (int i = 0; i < EXACT_MAXD; i++) {
      if (i + 1 < (int)D) {
        int64_t v = s[i] + c;
        c = v >> 32;
        s[i] = v - (c << 32);
      } else if (i + 1 == (int)D) {
        s[i] += c;
      }
    }
  }
  __device__ __forceinline__ bool zero() const {
    int64_t o = 0;
#pragma unroll
    for (int i = 0; i < EXACT_MAXD; i++) o |= s[i];
    return o == 0;
  }
};

// Round the exact value held in D slots (any carry state) to a double,
// nearest with ties to even.  Sets *overflow if the value does not fit the
// D-digit window.  The digits are carried into 32-bit words, the leading
// word and the two below it give a 96-bit window holding the 53 result
// bits, the rounding bit and the first sticky bits; words further down
// only feed the sticky bit.  Every index is resolved with unrolled selects.
__device__ inline double exact_round(const int64_t* slot, uint32_t D, int32_t lsb, uint32_t* overflow) {
  uint32_t dg[EXACT_MAXD];
  int64_t c = 0;
#pragma unroll
  for (int i = 0; i < EXACT_MAXD; i++) {
    dg[i] = 0;
    if (i < (int)D) {
      const int64_t v = slot[i] + c;
      c = v >> 32;
      dg[i] = (uint32_t)v;
    }
  }
  // c is the value above the top digit: it must be a sign extension
  if (c != 0 && c != -1 && overflow) *overflow = 1;
  const bool neg = c < 0;
  if (neg) {  // magnitude of the two's complement value
    uint64_t carry = 1;
#pragma unroll
    for (int i = 0; i < EXACT_MAXD; i++)
      if (i < (int)D) {
        const uint64_t v = (uint64_t)(uint32_t)~dg[i] + carry;
        dg[i] = (uint32_t)v;
        carry = v >> 32;
      }
  }
  int ti = -1;
#pragma unroll
  for (int i = 0; i < EXACT_MAXD; i++)
    if (dg[i]) ti = i;
  if (ti < 0) return 0.0;
  uint32_t d2 = 0, d1 = 0, d0 = 0;
  bool below = false;
#pragma unroll
  for (int i = 0; i < EXACT_MAXD; i++) {
    if (i == ti) d2 = dg[i];
    if (i == ti - 1) d1 = dg[i];
    if (i == ti - 2) d0 = dg[i];
    if (i < ti - 2 && dg[i]) below = true;
  }
  const int lz = __builtin_clz(d2);
  const uint64_t hi = ((uint64_t)d2 << 32) | d1;
  const uint64_t win = lz ? (hi << lz) | (d0 >> (32 - lz)) : hi;   // leading one at bit 63
  const uint32_t rest = lz ? d0 << lz : d0;
  uint64_t m = win >> 11;                                          // 53 bits
  const bool rbit = (win >> 10) & 1ull;
  const bool sticky = below || rest != 0 || (win & 0x3ffull) != 0;
  int e = ti * 32 + 31 - lz - 52 + lsb;
  if (rbit && (sticky || (m & 1ull))) {
    m++;
    if (m == (1ull << 53)) {
      m >>= 1;
      e++;
    }
  }
  const double r = ldexp((double)m, e);
  return neg ? -r : r;
}

}  // namespace lh
