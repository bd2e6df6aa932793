// Runs rocRAND's Philox4x32-10 engine (its public device API, compiled for the
// host) on counters read from stdin, one "seed c0 c1 c2 c3" line (hex) each,
// and prints the four output words. Used only as an independent reference
// for the oracle's Philox in tests; c1 must stay below 2^30 because the
// engine's offset argument counts 32-bit outputs in 64 bits.
#include <rocrand/rocrand_kernel.h>

#include <cstdio>

int main() {
  unsigned long long seed;
  unsigned c0, c1, c2, c3;
  while (std::scanf("%llx %x %x %x %x", &seed, &c0, &c1, &c2, &c3) == 5) {
    rocrand_state_philox4x32_10 st;
    const unsigned long long subsequence = (static_cast<unsigned long long>(c3) << 32) | c2;
    const unsigned long long offset = 4ull * ((static_cast<unsigned long long>(c1) << 32) | c0);
    rocrand_init(seed, subsequence, offset, &st);
    const uint4 v = rocrand4(&st);
    std::printf("%08x %08x %08x %08x\n", v.x, v.y, v.z, v.w);
  }
  return 0;
}
