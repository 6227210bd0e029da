// Exact, order-independent FP64 summation on the device.
//
// A sum of products is accumulated as a fixed-point integer whose least
// significant bit has weight 2^lsb, held in D 64-bit slots of 32-bit
// digits (slot i has weight 2^(lsb + 32 i)), and rounded once to the
// nearest double, ties to even.  Because integer addition is associative,
// the result does not depend on the order of the terms, the intersection
// algorithm, the set layout or the batching.
//
// A term v repeated mult times (mult < 2^64: rows of bag relations that
// carry no annotation) is split into the exact words of |v| * mult / 2^lsb,
// at most five 32-bit words, so every addition into a slot is below 2^32
// in magnitude whatever the multiplicity.
//
// Two slot forms exist:
//  - register accumulators (RegAcc) add signed words into int64 slots and
//    carry every 2^24 additions, so no slot leaves int64;
//  - shared accumulators (global or LDS, updated with atomics) keep every
//    slot below the top one as an unsigned value modulo 2^64.  An atomic
//    add returns the slot's previous value, from which the adding thread
//    knows exactly whether its own addition wrapped; it then adds the wrap
//    (+-2^32) into the next slot.  Atomic adds are linearizable, so the
//    wraps counted this way are exactly those of the serial history, and
//    the value is kept exactly for any number of additions.  The top slot
//    is signed; the plan sizes D so that it stays far inside int64.
// Both forms are read with the same carry rule (lower slots unsigned, top
// slot signed), since a normalized register accumulator is also a valid
// shared-form value.
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

// Multiply with saturation at UINT64_MAX (row multiplicities and counts).
__device__ __forceinline__ uint64_t sat_mul_u64(uint64_t a, uint64_t b) {
  const uint64_t hi = __umul64hi(a, b);
  return hi ? UINT64_MAX : a * b;
}
__device__ __forceinline__ uint64_t sat_add_u64(uint64_t a, uint64_t b) {
  const uint64_t s = a + b;
  return s < a ? UINT64_MAX : s;
}

// |v| * mult / 2^lsb as five 32-bit words p[0..4] placed at digit k0.
// Returns false when v has bits below 2^lsb.  v == 0 or mult == 0 gives
// all-zero words.
__device__ __forceinline__ bool term_words(double v, int32_t lsb, uint64_t mult, int32_t& k0, uint32_t* p,
                                           bool& neg) {
  const uint64_t bits = (uint64_t)__double_as_longlong(v);
  neg = (bits >> 63) != 0;
  const uint32_t ex = (uint32_t)(bits >> 52) & 0x7ffu;
  uint64_t mant = bits & ((1ull << 52) - 1);
  int32_t e;
  if (ex == 0) {
    e = -1074;
  } else {
    mant |= 1ull << 52;
    e = (int32_t)ex - 1075;
  }
#pragma unroll
  for (int j = 0; j < 5; j++) p[j] = 0;
  k0 = 0;
  if (mant == 0 || mult == 0) return true;
  int32_t sh = e - lsb;
  if (sh < 0) {
    const int tz = __builtin_ctzll(mant);
    if (tz < -sh) return false;
    mant >>= -sh;
    sh = 0;
  }
  k0 = sh >> 5;
  const uint32_t off = (uint32_t)sh & 31u;
  // the magnitude as three words: mant << off < 2^85
  const uint64_t lo = mant << off;                       // low 64 bits
  const uint64_t hi = off ? (mant >> (64 - off)) : 0;    // bits 64..84
  const uint32_t w[3] = {(uint32_t)lo, (uint32_t)(lo >> 32), (uint32_t)hi};
  if (mult == 1) {
    p[0] = w[0];
    p[1] = w[1];
    p[2] = w[2];
    return true;
  }
  const uint32_t m[2] = {(uint32_t)mult, (uint32_t)(mult >> 32)};
  // schoolbook product of 3 x 2 words; each partial sum stays below 2^64
#pragma unroll
  for (int i = 0; i < 3; i++) {
    uint64_t carry = 0;
#pragma unroll
    for (int j = 0; j < 2; j++) {
      const uint64_t t = (uint64_t)w[i] * m[j] + p[i + j] + carry;
      p[i + j] = (uint32_t)t;
      carry = t >> 32;
    }
    p[i + 2] = (uint32_t)carry;
  }
  return true;
}

// Register accumulator with a compile-time slot count; D <= EXACT_MAXD
// slots are live.  Dynamic digit indices are resolved with selects so the
// slots stay in registers.
struct RegAcc {
  int64_t s[EXACT_MAXD];
  uint32_t pending;   // additions since the last carry
  __device__ __forceinline__ void clear() {
#pragma unroll
    for (int i = 0; i < EXACT_MAXD; i++) s[i] = 0;
    pending = 0;
  }
  // Adds mult * v; returns false if v does not fit the window.
  __device__ __forceinline__ bool add(double v, int32_t lsb, uint32_t D, uint64_t mult) {
    if (v == 0.0) return true;
    int32_t k0;
    uint32_t p[5];
    bool neg;
    if (!term_words(v, lsb, mult, k0, p, neg)) return false;
    bool ok = true;
#pragma unroll
    for (int j = 0; j < 5; j++) ok = ok && (k0 + j < (int32_t)D || p[j] == 0);
#pragma unroll
    for (int i = 0; i < EXACT_MAXD; i++) {
      const uint32_t w = (i == k0) ? p[0] : (i == k0 + 1) ? p[1] : (i == k0 + 2) ? p[2] : (i == k0 + 3) ? p[3]
                       : (i == k0 + 4) ? p[4] : 0u;
      s[i] += neg ? -(int64_t)w : (int64_t)w;
    }
    // each addition is below 2^32 in magnitude: carry long before 2^63
    if (++pending >= (1u << 24)) normalize(D);
    return ok;
  }
  // Propagate carries so slots 0..D-2 hold digits in [0, 2^32) and the top
  // slot the signed rest.
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
    pending = 0;
  }
  // Take the value of shared-form slots (below the top: unsigned modulo
  // 2^64; top: signed), normalized.
  __device__ __forceinline__ void load_shared(const int64_t* slot, uint32_t D) {
    int64_t c = 0;
#pragma unroll
    for (int i = 0; i < EXACT_MAXD; i++) {
      s[i] = 0;
      if (i + 1 < (int)D) {
        const uint64_t u = (uint64_t)slot[i];
        const int64_t t = (int64_t)(u & 0xffffffffull) + c;
        s[i] = t & 0xffffffffll;
        c = (t >> 32) + (int64_t)(u >> 32);
      } else if (i + 1 == (int)D) {
        s[i] = slot[i] + c;
      }
    }
    pending = 0;
  }
  __device__ __forceinline__ bool zero() const {
    int64_t o = 0;
#pragma unroll
    for (int i = 0; i < EXACT_MAXD; i++) o |= s[i];
    return o == 0;
  }
};

// Atomically add the signed value v (|v| < 2^63) to slot q of a shared-form
// accumulator (global or LDS).  A wrap of a slot below the top moves +-2^32
// into the next slot, itself an atomic add that may wrap in turn.
__device__ __forceinline__ void atomic_add_digit(int64_t* slots, uint32_t q, uint32_t D, int64_t v) {
  while (v != 0 && q < D) {
    const uint64_t old = atomicAdd((unsigned long long*)&slots[q], (unsigned long long)v);
    if (q + 1 >= D) return;
    const uint64_t now = old + (uint64_t)v;
    int64_t carry = 0;
    if (v > 0 && now < old) carry = 1;
    else if (v < 0 && now > old) carry = -1;
    v = carry * (1ll << 32);
    q++;
  }
}

// Add a normalized register accumulator (or any slots whose lower values
// are non-negative) to a shared-form accumulator.
__device__ __forceinline__ void atomic_add_acc(int64_t* slots, const RegAcc& t, uint32_t D) {
  for (uint32_t q = 0; q < D; q++)
    if (t.s[q]) atomic_add_digit(slots, q, D, t.s[q]);
}

// Add mult * v straight into a shared-form accumulator: at most five
// atomics.  Returns false if v does not fit the window.
__device__ __forceinline__ bool atomic_add_term(int64_t* slots, double v, int32_t lsb, uint32_t D, uint64_t mult) {
  if (v == 0.0) return true;
  int32_t k0;
  uint32_t p[5];
  bool neg;
  if (!term_words(v, lsb, mult, k0, p, neg)) return false;
  bool ok = true;
#pragma unroll
  for (int j = 0; j < 5; j++) {
    if (!p[j]) continue;
    if (k0 + j >= (int32_t)D) {
      ok = false;
      continue;
    }
    atomic_add_digit(slots, (uint32_t)(k0 + j), D, neg ? -(int64_t)p[j] : (int64_t)p[j]);
  }
  return ok;
}

// Round the exact value held in D shared-form slots (a normalized register
// accumulator is one too) to a double, nearest with ties to even.  Sets
// *overflow if the value does not fit the D-digit window.  The slots are
// carried into 32-bit words, the leading word and the two below it give a
// 96-bit window holding the 53 result bits, the rounding bit and the first
// sticky bits; words further down only feed the sticky bit.  Every index is
// resolved with unrolled selects.
__device__ inline double exact_round(const int64_t* slot, uint32_t D, int32_t lsb, uint32_t* overflow) {
  uint32_t dg[EXACT_MAXD];
  int64_t c = 0;
#pragma unroll
  for (int i = 0; i < EXACT_MAXD; i++) {
    dg[i] = 0;
    if (i + 1 < (int)D) {
      const uint64_t u = (uint64_t)slot[i];
      const int64_t t = (int64_t)(u & 0xffffffffull) + c;
      dg[i] = (uint32_t)t;
      c = (t >> 32) + (int64_t)(u >> 32);
    } else if (i + 1 == (int)D) {
      const int64_t v = slot[i] + c;
      dg[i] = (uint32_t)v;
      c = v >> 32;
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

// The exact value held in D shared-form slots as parts out[0..K): each part
// is the nearest double to what the parts before it leave, so out[0] is
// the correctly rounded sum, the parts do not overlap, and their exact sum
// is the value whenever K parts suffice (each part takes at least 53 of the
// value's 32 D bits: K = 5 covers D = 8).  Unused parts are 0.  Sets
// *overflow if the value does not fit the window or K parts do not suffice.
constexpr int EXACT_PARTS = 5;
__device__ inline void exact_parts(const int64_t* slot, uint32_t D, int32_t lsb, double* out, uint32_t* overflow) {
  RegAcc r;
  r.load_shared(slot, D);
  bool done = false;
#pragma unroll
  for (int k = 0; k < EXACT_PARTS; k++) {
    double v = 0.0;
    if (!done) {
      v = exact_round(r.s, D, lsb, overflow);
      if (v == 0.0) {
        done = true;
      } else {
        // v is a multiple of 2^lsb inside the window: the subtraction is exact
        (void)r.add(-v, lsb, D, 1);
        r.normalize(D);
      }
    }
    out[k] = v;
  }
  if (!done && !r.zero() && overflow) *overflow = 1;
}

}  // namespace lh
