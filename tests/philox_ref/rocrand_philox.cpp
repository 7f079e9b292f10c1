// Reads "c0 c1 c2 c3 k0 k1" lines and prints the Philox4x32-10 block computed
// by rocRAND's engine (host build).  rocRAND maps (seed, subsequence, offset)
// to key = seed, counter words 2..3 = subsequence, counter words 0..1 =
// offset / 4 (offset counts 32-bit outputs); four calls return words 0..3.
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>

int main() {
  unsigned long long c0, c1, c2, c3, k0, k1;
  while (std::scanf("%llu %llu %llu %llu %llu %llu", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
    rocrand_device::philox4x32_10_engine eng(k0 | (k1 << 32), c2 | (c3 << 32), 0);
    // advance c1 * 2^32 + c0 blocks without overflowing the 64-bit output offset
    for (int i = 0; i < 4; ++i) eng.discard(c1 << 32);
    eng.discard(4 * c0);
    unsigned w0 = eng(), w1 = eng(), w2 = eng(), w3 = eng();
    std::printf("%u %u %u %u\n", w0, w1, w2, w3);
  }
  return 0;
}
