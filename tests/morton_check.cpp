// Host check of the Morton helpers the kernels use: the displaced-key step
// (interleaved carry and borrow) against decode, add modulo 2^bits, encode,
// for every grid size 2^0 .. 2^21 per axis and all 27 offsets.
#include "../paper_0904_3662_amd/csrc/ahf_dev.h"

#include <cstdio>
#include <random>

using namespace ahf;

static uint64_t by_coordinates(uint64_t k, int bits, int dx, int dy, int dz) {
  uint32_t x, y, z;
  unmorton3(k, x, y, z);
  const uint32_t m = (1u << bits) - 1u;
  return morton3((uint32_t)((int32_t)x + dx) & m, (uint32_t)((int32_t)y + dy) & m,
                 (uint32_t)((int32_t)z + dz) & m);
}

int main() {
  std::mt19937_64 rng(7);
  long bad = 0, n = 0;
  for (int bits = 0; bits <= 21; ++bits) {
    const uint64_t mask = (1ull << (3 * bits)) - 1ull;
    const uint32_t e = (1u << bits) - 1u;
    for (int it = 0; it < 4000; ++it) {
      // the 8 corners of the grid first, then random cells
      const uint64_t k = it < 8 ? morton3(it & 1 ? e : 0, it & 2 ? e : 0, it & 4 ? e : 0)
                                : (rng() & mask);
      if (morton3(0, 0, 0) != 0 || by_coordinates(k, bits, 0, 0, 0) != k) ++bad;
      for (int o = 0; o < 27; ++o, ++n) {
        const int dx = o / 9 - 1, dy = (o / 3) % 3 - 1, dz = o % 3 - 1;
        if (shift_key(k, bits, dx, dy, dz) != by_coordinates(k, bits, dx, dy, dz)) ++bad;
      }
    }
  }
  std::printf("%ld mismatches of %ld\n", bad, n);
  return bad != 0;
}
