// Runs the device exact accumulator's arithmetic on the host.
// stdin: "D lsb" then "s0 .. s{D-1}" (initial shared slots, unsigned
// decimal), then lines "mode v_bits mult" until EOF: mode 0 adds mult * v to
// a register accumulator (flushed into the shared slots at the end), mode 1
// adds it straight to the shared slots.  stdout: "ok overflow bits" where
// bits is the rounded sum's IEEE pattern and ok is 0 if a term did not fit,
// then the IEEE patterns of the value's exact parts (exact_parts).
#include <stdio.h>
#include <stdlib.h>

#include "../../paper_1708_07859_amd/csrc/exact.h"

int main() {
  unsigned D;
  int lsb;
  if (scanf("%u %d", &D, &lsb) != 2) return 2;
  int64_t slots[lh::EXACT_MAXD] = {0};
  for (unsigned i = 0; i < D; i++) {
    unsigned long long u;
    if (scanf("%llu", &u) != 1) return 2;
    slots[i] = (int64_t)u;
  }
  lh::RegAcc acc;
  acc.clear();
  bool ok = true;
  int mode;
  unsigned long long vb, mult;
  while (scanf("%d %llu %llu", &mode, &vb, &mult) == 3) {
    double v;
    memcpy(&v, &vb, sizeof v);
    if (mode == 0) ok = acc.add(v, lsb, D, mult) && ok;
    else ok = lh::atomic_add_term(slots, v, lsb, D, mult) && ok;
  }
  acc.normalize(D);
  lh::atomic_add_acc(slots, acc, D);
  uint32_t ovf = 0;
  const double r = lh::exact_round(slots, D, lsb, &ovf);
  unsigned long long rb;
  memcpy(&rb, &r, sizeof rb);
  double parts[lh::EXACT_PARTS];
  uint32_t povf = 0;
  lh::exact_parts(slots, D, lsb, parts, &povf);
  printf("%d %u %llu", ok ? 1 : 0, ovf | povf, rb);
  for (int k = 0; k < lh::EXACT_PARTS; k++) {
    unsigned long long pb;
    memcpy(&pb, &parts[k], sizeof pb);
    printf(" %llu", pb);
  }
  printf("\n");
  return 0;
}
