// Host check of the closed-form tile count used by the prefix scans: it must
// equal the bucket-by-bucket count (every bucket below the size contributes
// ceil(live elements / tile) tiles) for every first-bucket size 2^0..2^19, every
// tile size 2^10..2^14, all sizes below 5000, bucket boundaries +-1 and random
// sizes up to 2^44.  Prints "ok <cases>" or the first mismatch (exit 1).
#include "gga_internal.h"
#include <cstdio>
#include <random>
static uint64_t loop(uint32_t f, uint64_t s, uint32_t k) {
  uint64_t n = 0;
  const uint32_t nb = gga::nbuckets_for(f, s);
  for (uint32_t b = 0; b < nb; ++b) {
    const uint64_t st = gga::bucket_start(f, b);
    uint64_t live = gga::bucket_len(f, b);
    if (s - st < live) live = s - st;
    n += (live + (1ull << k) - 1) >> k;
  }
  return n;
}
int main() {
  std::mt19937_64 rng(5);
  uint64_t cnt = 0;
  for (uint32_t f = 0; f < 20; ++f)
    for (uint32_t k = 10; k <= 14; ++k) {
      for (uint64_t s = 0; s < 5000; ++s, ++cnt)
        if (loop(f, s, k) != gga::tiles_for(f, s, k)) { printf("mismatch f=%u k=%u s=%llu\n", f, k, (unsigned long long)s); return 1; }
      for (int i = 0; i < 20000; ++i, ++cnt) {
        const uint64_t s = rng() >> (20 + (rng() & 15));
        if (loop(f, s, k) != gga::tiles_for(f, s, k)) { printf("mismatch f=%u k=%u s=%llu\n", f, k, (unsigned long long)s); return 1; }
      }
      for (uint32_t b = 0; b < 36; ++b)
        for (int d = -1; d <= 1; ++d, ++cnt) {
          const uint64_t s = gga::bucket_start(f, b) + d;
          if ((int64_t)s < 0) continue;
          if (loop(f, s, k) != gga::tiles_for(f, s, k)) { printf("mismatch f=%u k=%u s=%llu\n", f, k, (unsigned long long)s); return 1; }
        }
    }
  printf("ok %llu\n", (unsigned long long)cnt);
  return 0;
}
