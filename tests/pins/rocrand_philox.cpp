// Library cross-check for the oracle's Philox4x32-10: evaluates the block
// function through rocRAND's header-only philox4x32_10 engine on the host.
// Input lines: key0 key1 c0 c1 c2 c3 (decimal uint32); output: four words.
// The engine's counter is (x, y) = offset / 4 and (z, w) = subsequence, its
// key is the 64-bit seed, so any (counter, key) pair can be reached.
#include <rocrand/rocrand_kernel.h>
#include <cstdio>
#include <cstdint>

int main() {
  unsigned long long k0, k1, c0, c1, c2, c3;
  while (std::scanf("%llu %llu %llu %llu %llu %llu", &k0, &k1, &c0, &c1, &c2,
                    &c3) == 6) {
    unsigned long long seed = k0 | (k1 << 32);
    unsigned long long subsequence = c2 | (c3 << 32);
    unsigned long long block = c0 | (c1 << 32);
    rocrand_device::philox4x32_10_engine eng(seed, subsequence, 0ull);
    // offset counts 32-bit outputs; advance by whole blocks, possibly 2^64+.
    // Split the 4*block skip so that it never overflows 64 bits.
    for (int part = 0; part < 4; ++part) eng.discard(block);
    unsigned w0 = eng.next(), w1 = eng.next(), w2 = eng.next(), w3 = eng.next();
    std::printf("%u %u %u %u\n", w0, w1, w2, w3);
  }
  return 0;
}
