// Independent witness for the oracle's Philox4x32-10: evaluates the generator
// through rocRAND's published engine (host side) for counters read on stdin.
// Input lines: c0 c1 c2 c3 k0 k1 (hex); output: four hex words.
// The engine is positioned so that its next block uses counter (c0, c1, c2, c3):
// subsequence = (c3 << 32) | c2 fills counter words 2-3, and an offset of
// 4 * ((c1 << 32) | c0) draws fills words 0-1 (requires c1 < 2^30).
#include <cstdio>
#include <rocrand/rocrand_philox4x32_10.h>

int main() {
  unsigned c0, c1, c2, c3, k0, k1;
  while (std::scanf("%x %x %x %x %x %x", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
    if (c1 >= (1u << 30)) return 2;
    unsigned long long seed = ((unsigned long long)k1 << 32) | k0;
    unsigned long long subsequence = ((unsigned long long)c3 << 32) | c2;
    unsigned long long offset = 4ull * (((unsigned long long)c1 << 32) | c0);
    rocrand_device::philox4x32_10_engine engine(seed, subsequence, offset);
    uint4 r = engine.next4();
    std::printf("%08x %08x %08x %08x\n", r.x, r.y, r.z, r.w);
  }
  return 0;
}
