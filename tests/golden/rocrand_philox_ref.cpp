// Independent Philox4x32-10 for cross-checking: rocRAND's engine, built for
// the host only (no GPU is touched).  Reads lines "seed k b" (decimal or
// 0x-hex) and prints the four 32-bit words of block (k, b) under key seed.
// rocRAND's engine(seed, subsequence, offset) uses key = (seed lo, seed hi),
// counter words z,w = subsequence and counter words x,y = offset / 4, so
// counter (k lo, k hi, b, 0) is engine(seed, b, 4k) for k < 2^62.
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>
#include <cstdlib>
int main() {
  char a[64], b[64], c[64];
  while (std::scanf("%63s %63s %63s", a, b, c) == 3) {
    unsigned long long seed = std::strtoull(a, nullptr, 0);
    unsigned long long k = std::strtoull(b, nullptr, 0);
    unsigned long long blk = std::strtoull(c, nullptr, 0);
    rocrand_device::philox4x32_10_engine e(seed, blk, 4ull * k);
    unsigned int w0 = e(), w1 = e(), w2 = e(), w3 = e();
    std::printf("%u %u %u %u\n", w0, w1, w2, w3);
  }
  return 0;
}
