// Test helper: prints the four words of ATen's open-source Philox4_32 engine
// (torch/include/ATen/core/PhiloxRNGEngine.h) for each "seed subsequence
// offset" line read from stdin.  A third, independent Philox4x32-10 used to
// cross-check the oracle's generator and its counter layout; never linked
// into the product.
#include <ATen/core/PhiloxRNGEngine.h>

#include <cinttypes>
#include <cstdio>

int main() {
  unsigned long long seed, sub, off;
  while (std::scanf("%llu %llu %llu", &seed, &sub, &off) == 3) {
    at::Philox4_32 engine(seed, sub, off);
    uint32_t w0 = engine(), w1 = engine(), w2 = engine(), w3 = engine();
    std::printf("%" PRIu32 " %" PRIu32 " %" PRIu32 " %" PRIu32 "\n", w0, w1, w2, w3);
  }
  return 0;
}
