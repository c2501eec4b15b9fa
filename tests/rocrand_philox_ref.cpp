// Test helper: prints Philox4x32-10 blocks computed by the installed rocRAND
// engine (host-callable header), for counters and keys read from stdin as
// "c0 c1 c2 c3 k0 k1" lines (decimal).  Used only to pin the oracle's Philox.
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>

int main() {
  unsigned long long c0, c1, c2, c3, k0, k1;
  while (std::scanf("%llu %llu %llu %llu %llu %llu", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
    unsigned long long seed = k0 | (k1 << 32);
    unsigned long long blocks = c0 | (c1 << 32);   // counter words 0-1
    unsigned long long subsequence = c2 | (c3 << 32);  // counter words 2-3
    rocrand_device::philox4x32_10_engine eng(seed, subsequence, 0);
    while (blocks > 0) {  // skip whole blocks in chunks that fit the 64-bit offset
      unsigned long long chunk = blocks < (1ULL << 60) ? blocks : (1ULL << 60);
      eng.discard(4ULL * chunk);
      blocks -= chunk;
    }
    unsigned int a = eng.next(), b = eng.next(), c = eng.next(), d = eng.next();
    std::printf("%u %u %u %u\n", a, b, c, d);
  }
  return 0;
}
