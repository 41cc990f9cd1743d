// Host-only driver of rocRAND's Philox4x32-10 block function, used by
// tests/test_oracle_philox_rocrand.py as an implementation of the generator
// that is independent of the oracle.  Reads lines "c0 c1 c2 c3 k0 k1"
// (decimal uint32) on stdin and prints the four output words of the block at
// counter (c0, c1, c2, c3) under key (k0, k1).
//
// The block function (ten rounds with key bumps) is a protected member of
// rocRAND's engine; a derived class exposes it, so any counter, including
// ones the engine's seek interface cannot reach in one call, can be probed.
#include <cstdio>

#include <rocrand/rocrand_philox4x32_10.h>

struct PhiloxBlock : rocrand_device::philox4x32_10_engine {
  uint4 block(uint4 ctr, uint2 key) { return ten_rounds(ctr, key); }
};

int main() {
  unsigned int c[4], k[2];
  PhiloxBlock eng;
  while (std::scanf("%u %u %u %u %u %u", &c[0], &c[1], &c[2], &c[3], &k[0], &k[1]) == 6) {
    uint4 ctr;
    ctr.x = c[0];
    ctr.y = c[1];
    ctr.z = c[2];
    ctr.w = c[3];
    uint2 key;
    key.x = k[0];
    key.y = k[1];
    const uint4 r = eng.block(ctr, key);
    std::printf("%u %u %u %u\n", r.x, r.y, r.z, r.w);
  }
  return 0;
}
