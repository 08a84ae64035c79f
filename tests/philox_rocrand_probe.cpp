// Host-only probe: prints rocRAND's Philox4x32-10 block for (seed, counter).
// Used by the oracle's CPU tests as an independent library implementation.
// Input lines: seed c0 c1 c2 c3 ; output lines: the four 32-bit words.
#include <rocrand/rocrand_philox4x32_10.h>

#include <cstdio>

int main() {
  unsigned long long seed;
  unsigned c0, c1, c2, c3;
  while (std::scanf("%llu %u %u %u %u", &seed, &c0, &c1, &c2, &c3) == 5) {
    rocrand_state_philox4x32_10 st;
    // rocRAND: subsequence adds to counter words 2,3; offset/4 adds to words 0,1.
    unsigned long long subseq = (static_cast<unsigned long long>(c3) << 32) | c2;
    unsigned long long offset = 4ull * ((static_cast<unsigned long long>(c1) << 32) | c0);
    rocrand_init(seed, subseq, offset, &st);
    uint4 r = rocrand4(&st);
    std::printf("%u %u %u %u\n", r.x, r.y, r.z, r.w);
  }
  return 0;
}
