// Independent Philox4x32-10 reference for the oracle's generator: PyTorch's
// header-only at::philox_engine.  Its counter is (offset lo, offset hi,
// subsequence lo, subsequence hi) and its key is (seed lo, seed hi), so any
// (counter, key) pair can be set through the constructor.  Reads lines
// "c0 c1 c2 c3 k0 k1" and prints the four output words of each.
#include <ATen/core/PhiloxRNGEngine.h>

#include <cinttypes>
#include <cstdio>

int main() {
  unsigned long long c0, c1, c2, c3, k0, k1;
  while (std::scanf("%llu %llu %llu %llu %llu %llu", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
    uint64_t seed = (uint64_t)k0 | ((uint64_t)k1 << 32);
    uint64_t subseq = (uint64_t)c2 | ((uint64_t)c3 << 32);
    uint64_t offset = (uint64_t)c0 | ((uint64_t)c1 << 32);
    at::philox_engine e(seed, subseq, offset);
    uint32_t w0 = e(), w1 = e(), w2 = e(), w3 = e();
    std::printf("%u %u %u %u\n", w0, w1, w2, w3);
  }
  return 0;
}
