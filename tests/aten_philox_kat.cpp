// Known-answer source for Philox-4x32-10: PyTorch's own host implementation
// (ATen/core/PhiloxRNGEngine.h), compiled and run by a test.  Reads lines
// "seed subsequence offset" and prints the first four 32-bit outputs, i.e.
// Philox((offset_lo, offset_hi, subseq_lo, subseq_hi), (seed_lo, seed_hi)).
#include <ATen/core/PhiloxRNGEngine.h>
#include <cstdio>

int main() {
  unsigned long long seed, sub, off;
  while (std::scanf("%llu %llu %llu", &seed, &sub, &off) == 3) {
    at::philox_engine e(seed, sub, off);
    unsigned a = e(), b = e(), c = e(), d = e();
    std::printf("%u %u %u %u\n", a, b, c, d);
  }
  return 0;
}
