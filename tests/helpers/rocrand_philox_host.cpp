// Host-only helper for the CPU tests: evaluates single Philox4x32-10 blocks with
// rocRAND's engine (an independent library implementation) so the oracle's
// block function can be checked against it.  Reads "c0 c1 c2 c3 k0 k1" lines
// (hex) from stdin and prints the four output words.
#include <cstdio>
#include <rocrand/rocrand_philox4x32_10.h>

int main() {
  unsigned c[4], k[2];
  while (std::scanf("%x %x %x %x %x %x", &c[0], &c[1], &c[2], &c[3], &k[0], &k[1]) == 6) {
    // rocRAND places the seed in the key, the subsequence in counter words 2-3
    // and offset/4 in counter words 0-1.
    unsigned long long seed = (unsigned long long)k[0] | ((unsigned long long)k[1] << 32);
    unsigned long long subseq = (unsigned long long)c[2] | ((unsigned long long)c[3] << 32);
    unsigned long long block = (unsigned long long)c[0] | ((unsigned long long)c[1] << 32);
    rocrand_device::philox4x32_10_engine eng(seed, subseq, 0);
    // discard() takes an offset in words (4 per block); split it so it cannot wrap.
    const unsigned long long q = block >> 2, rem = block & 3ull;
    for (int i = 0; i < 4; ++i) eng.discard(q * 4ull);
    eng.discard(rem * 4ull);
    uint4 r = eng.next4();
    std::printf("%08x %08x %08x %08x\n", r.x, r.y, r.z, r.w);
  }
  return 0;
}
