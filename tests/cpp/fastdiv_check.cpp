// Host check of txs::FastDiv (the multiply-high division by a launch-time
// divisor used to map points to rays): against plain unsigned division for
// all divisors 1..4096 on edge and random numerators, and for random
// divisors up to 2^32-1.  Prints "ok" or the first mismatch.
#include <cstdint>
#include <cstdio>
#include <random>

#include "txs_common.h"

static bool check(uint32_t d, uint32_t n) {
  const txs::FastDiv f(d);
  if (f.div(n) != n / d) {
    std::printf("mismatch d=%u n=%u got=%u want=%u\n", d, n, f.div(n), n / d);
    return false;
  }
  return true;
}

int main() {
  std::mt19937_64 rng(12345);
  const uint32_t edge[] = {0u, 1u, 2u, 3u, 127u, 128u, 129u, 65535u, 65536u, 0x7fffffffu,
                           0x80000000u, 0xfffffffeu, 0xffffffffu};
  for (uint32_t d = 1; d <= 4096; ++d) {
    for (uint32_t n : edge)
      if (!check(d, n)) return 1;
    for (uint32_t m = 1; m < 64; ++m) {  // around multiples of d
      const uint64_t q = (uint64_t)rng() % (0xffffffffull / d + 1);
      for (int64_t off = -1; off <= 1; ++off) {
        const int64_t n = (int64_t)(q * d) + off;
        if (n >= 0 && n <= 0xffffffffll && !check(d, (uint32_t)n)) return 1;
      }
    }
    for (int i = 0; i < 200; ++i)
      if (!check(d, (uint32_t)rng())) return 1;
  }
  for (int i = 0; i < 20000; ++i) {
    const uint32_t d = 1u + (uint32_t)(rng() % 0xffffffffull);
    for (uint32_t n : edge)
      if (!check(d, n)) return 1;
    for (int j = 0; j < 20; ++j)
      if (!check(d, (uint32_t)rng())) return 1;
  }
  std::printf("ok\n");
  return 0;
}
