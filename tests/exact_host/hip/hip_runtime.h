// Host stand-in for the few HIP device builtins the exact accumulator uses,
// so that its arithmetic can be checked on the CPU.  Atomics act on one
// thread: each returns the previous value, as the device's do.
#pragma once
#include <math.h>
#include <stdint.h>
#include <string.h>

#define __device__
#define __forceinline__ inline

inline long long __double_as_longlong(double v) {
  long long b;
  memcpy(&b, &v, sizeof b);
  return b;
}
inline uint64_t __umul64hi(uint64_t a, uint64_t b) { return (uint64_t)(((unsigned __int128)a * b) >> 64); }
inline double __dmul_rn(double a, double b) { return a * b; }
inline double __fma_rn(double a, double b, double c) { return fma(a, b, c); }
inline unsigned long long atomicAdd(unsigned long long* p, unsigned long long v) {
  const unsigned long long old = *p;
  *p = old + v;
  return old;
}
template <class T>
inline T min(T a, T b) { return a < b ? a : b; }
