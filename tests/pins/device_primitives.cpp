// Host build of the GPU library's device primitives (de_device.hpp), so the
// CPU suite can compare them with the independent FP64 oracle and NumPy.
// Usage: device_primitives MODE < input; one query per line, one answer per
// line.  MODE: philox | donors | mask | xover | sin2 | mutant | key | xcd.
#include <cstdio>
#include <cstdint>
#include <cstring>
#include <vector>

#include "de_device.hpp"

static float f_of_bits(unsigned b) {
  float f;
  std::memcpy(&f, &b, 4);
  return f;
}
static unsigned bits_of(float f) {
  unsigned b;
  std::memcpy(&b, &f, 4);
  return b;
}

int main(int argc, char** argv) {
  if (argc < 2) return 2;
  const char* mode = argv[1];
  if (!std::strcmp(mode, "philox")) {
    unsigned k0, k1, c0, c1, c2, c3;
    while (std::scanf("%u %u %u %u %u %u", &k0, &k1, &c0, &c1, &c2, &c3) == 6) {
      const de::Words4 w = de::philox4x32_10(c0, c1, c2, c3, k0, k1);
      std::printf("%u %u %u %u\n", w.w[0], w.w[1], w.w[2], w.w[3]);
    }
  } else if (!std::strcmp(mode, "donors")) {
    unsigned long long seed;
    unsigned run, gen;
    int i, NP, D;
    while (std::scanf("%llu %u %u %d %d %d", &seed, &run, &gen, &i, &NP, &D) == 6) {
      const de::Donors d = de::pick_donors(run, gen, i, NP, D, (uint32_t)seed,
                                           (uint32_t)(seed >> 32));
      std::printf("%d %d %d %d\n", d.r1, d.r2, d.r3, d.jrand);
    }
  } else if (!std::strcmp(mode, "mask")) {
    // seed run gen i D jrand threshold -> D characters '0'/'1'
    unsigned long long seed;
    unsigned run, gen, thr;
    int i, D, jrand;
    while (std::scanf("%llu %u %u %d %d %d %u", &seed, &run, &gen, &i, &D, &jrand,
                      &thr) == 7) {
      std::vector<char> out(D + 1, 0);
      for (int q = 0; 4 * q < D; ++q) {
        const de::Words4 w = de::draw_block(de::kTagXover, run, gen, (uint32_t)i,
                                            (uint32_t)q, (uint32_t)seed,
                                            (uint32_t)(seed >> 32));
        for (int b = 0; b < 4 && 4 * q + b < D; ++b)
          out[4 * q + b] = de::take_mutant(w.w[b], 4 * q + b, jrand, thr) ? '1' : '0';
      }
      std::printf("%s\n", out.data());
    }
  } else if (!std::strcmp(mode, "xover")) {
    // word threshold -> 1 if the crossover test takes the mutant (j != jrand)
    unsigned w, thr;
    while (std::scanf("%u %u", &w, &thr) == 2)
      std::printf("%d\n", de::take_mutant(w, 0, 1, thr) ? 1 : 0);
  } else if (!std::strcmp(mode, "sin2")) {
    unsigned b;
    while (std::scanf("%u", &b) == 1)
      std::printf("%u\n", bits_of(de::sin_squared(f_of_bits(b))));
  } else if (!std::strcmp(mode, "mutant")) {
    unsigned a, b, c, F, lo, hi;
    while (std::scanf("%u %u %u %u %u %u", &a, &b, &c, &F, &lo, &hi) == 6)
      std::printf("%u\n", bits_of(de::mutant_coord(f_of_bits(a), f_of_bits(b),
                                                   f_of_bits(c), f_of_bits(F),
                                                   f_of_bits(lo), f_of_bits(hi))));
  } else if (!std::strcmp(mode, "key")) {
    unsigned b;
    int idx;
    while (std::scanf("%u %d", &b, &idx) == 2)
      std::printf("%llu\n", de::fit_key(f_of_bits(b), idx));
  } else if (!std::strcmp(mode, "xcd")) {
    int n;
    while (std::scanf("%d", &n) == 1) {
      std::vector<int> seen(n, 0);
      bool ok = true;
      for (int b = 0; b < n; ++b) {
        const int l = de::xcd_logical_block(b, n);
        if (l < 0 || l >= n || seen[l]++) ok = false;
      }
      std::printf("%s\n", ok ? "ok" : "bad");
    }
  } else {
    return 2;
  }
  return 0;
}
