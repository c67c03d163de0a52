// Test-only harness: evaluates PyTorch's independently written Philox4x32-10
// engine (ATen/core/PhiloxRNGEngine.h, header source) on raw (counter, key)
// pairs read from stdin, one "c0 c1 c2 c3 k0 k1" line per block, and prints
// the four output words.  The engine's seed is the key (low word first), its
// subsequence fills counter words 2-3 and its offset counter words 0-1.
#include <ATen/core/PhiloxRNGEngine.h>
#include <cstdint>
#include <cstdio>

int main() {
  unsigned long c0, c1, c2, c3, k0, k1;
  while (std::scanf("%lu %lu %lu %lu %lu %lu", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
    uint64_t seed = (uint64_t)k0 | ((uint64_t)k1 << 32);
    uint64_t subseq = (uint64_t)c2 | ((uint64_t)c3 << 32);
    uint64_t offset = (uint64_t)c0 | ((uint64_t)c1 << 32);
    at::Philox4_32 eng(seed, subseq, offset);
    uint32_t a = eng(), b = eng(), c = eng(), d = eng();
    std::printf("%u %u %u %u\n", a, b, c, d);
  }
  return 0;
}
