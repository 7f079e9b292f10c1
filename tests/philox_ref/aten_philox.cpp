// Reads "c0 c1 c2 c3 k0 k1" lines and prints the Philox4x32-10 block computed
// by PyTorch's ATen engine.  ATen maps (seed, subsequence, offset) to
// key = seed, counter words 2..3 = subsequence, counter words 0..1 = offset
// (in 128-bit blocks); four calls return output words 0..3.
#include <ATen/core/PhiloxRNGEngine.h>
#include <cstdint>
#include <cstdio>

int main() {
  unsigned long long c0, c1, c2, c3, k0, k1;
  while (std::scanf("%llu %llu %llu %llu %llu %llu", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
    at::Philox4_32 eng(k0 | (k1 << 32), c2 | (c3 << 32), c0 | (c1 << 32));
    uint32_t w0 = eng(), w1 = eng(), w2 = eng(), w3 = eng();
    std::printf("%u %u %u %u\n", w0, w1, w2, w3);
  }
  return 0;
}
