// Host-only program: prints Philox4x32-10 output blocks computed by rocRAND's
// open-source engine (an implementation independent of this repository).
// Input on stdin: lines "c0 c1 c2 c3 k0 k1" (decimal); output: four words.
// rocRAND's engine keys with the 64-bit seed (k0 | k1 << 32), places the
// subsequence in counter words 2-3 and offset/4 in counter words 0-1.
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>

int main() {
  unsigned long long c0, c1, c2, c3, k0, k1;
  while (std::scanf("%llu %llu %llu %llu %llu %llu", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
    unsigned long long seed = k0 | (k1 << 32);
    unsigned long long subseq = c2 | (c3 << 32);
    unsigned long long offset = 4ull * (c0 | (c1 << 32));
    rocrand_device::philox4x32_10_engine eng(seed, subseq, offset);
    unsigned int w[4];
    for (int j = 0; j < 4; ++j) w[j] = eng.next();
    std::printf("%u %u %u %u\n", w[0], w[1], w[2], w[3]);
  }
  return 0;
}
