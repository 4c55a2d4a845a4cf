// Independent Philox4x32-10 reference: rocRAND's engine run on the host.
// Reads lines "seed c0 c1 c2 c3" (decimal) on stdin and prints the four output
// words of the block at that counter.  rocRAND addresses a block by
// (subsequence = c2 | c3 << 32, offset = 4 * (c0 | c1 << 32)).
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>
int main() {
  unsigned long long seed, c0, c1, c2, c3;
  while (std::scanf("%llu %llu %llu %llu %llu", &seed, &c0, &c1, &c2, &c3) == 5) {
    rocrand_device::philox4x32_10_engine eng(seed, c2 | (c3 << 32), 4ull * (c0 | (c1 << 32)));
    unsigned a = eng.next(), b = eng.next(), c = eng.next(), d = eng.next();
    std::printf("%u %u %u %u\n", a, b, c, d);
  }
  return 0;
}
