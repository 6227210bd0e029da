// Runs the device search helpers of csrc/search.h on the host.
// stdin: n, the n sorted keys, q, then q queries "b e x";
// stdout per query: count_le_quinary(keys + b, e - b, x) and
// lower_bound_sampled_quinary(keys, samples, b, e, x).
#include <cstdio>
#include <vector>

#include "../../paper_1708_07859_amd/csrc/search.h"
using namespace lh;

int main() {
  unsigned n = 0, q = 0;
  if (scanf("%u", &n) != 1) return 1;
  std::vector<uint32_t> keys(n + 1), samp(n / 32 + 2);
  for (unsigned i = 0; i < n; i++)
    if (scanf("%u", &keys[i]) != 1) return 1;
  for (unsigned j = 0; j * 32 < n; j++) samp[j] = keys[j * 32];
  if (scanf("%u", &q) != 1) return 1;
  for (unsigned i = 0; i < q; i++) {
    unsigned b, e, x;
    if (scanf("%u %u %u", &b, &e, &x) != 3) return 1;
    const uint32_t c = count_le_quinary(keys.data() + b, e - b, x);
    const uint32_t lb = lower_bound_sampled_quinary(keys.data(), samp.data(), b, e, x);
    printf("%u %u\n", c, lb);
  }
  return 0;
}
