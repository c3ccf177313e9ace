// Independent Philox4x32-10 reference for the test suite: rocRAND's host-callable engine.
// Prints the 4 output words for each counter/key line read from stdin
// ("c0 c1 c2 c3 k0 k1" in decimal).  rocRAND's engine maps (seed, subsequence, offset) to
// key = seed, counter = (offset/4 as 64-bit in words 0-1, subsequence in words 2-3).
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>
#include <cstdint>
int main() {
  unsigned long long c0, c1, c2, c3, k0, k1;
  while (std::scanf("%llu %llu %llu %llu %llu %llu", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
    unsigned long long seed = k0 | (k1 << 32);
    unsigned long long subseq = c2 | (c3 << 32);
    unsigned long long offset = 4ull * (c0 | (c1 << 32));
    rocrand_device::philox4x32_10_engine eng(seed, subseq, offset);
    uint4 w = eng.next4();
    std::printf("%u %u %u %u\n", w.x, w.y, w.z, w.w);
  }
  return 0;
}
