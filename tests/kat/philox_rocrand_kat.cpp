// Known-answer source for Philox4x32-10 that is independent of the oracle:
// the open-source rocRAND generator header, run on the host.  Reads lines
// "seed stream step path" and prints the four 32-bit words of the block whose
// counter is (step, path, stream, 0) under key (seed_lo, seed_hi).
// rocRAND's state counter is (offset/4 as a 64-bit number over words 0-1) +
// (subsequence as a 64-bit number over words 2-3), so that block is reached
// with subsequence = stream and offset = 4 * (step + 2^32 * path).
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>

int main() {
  unsigned long long seed, stream, step, path;
  while (std::scanf("%llu %llu %llu %llu", &seed, &stream, &step, &path) == 4) {
    rocrand_state_philox4x32_10 st;
    rocrand_init(seed, stream, 4ull * (step + (path << 32)), &st);
    uint4 r = rocrand4(&st);
    std::printf("%u %u %u %u\n", r.x, r.y, r.z, r.w);
  }
  return 0;
}
