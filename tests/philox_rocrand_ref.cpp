// Philox4x32-10 reference outputs from rocRAND's open-source engine, run on
// the host.  Reads lines "c0 c1 c2 c3 k0 k1" (hex) and prints the four output
// words (hex) of ten rounds applied to that counter under that key.
// Test infrastructure: pins the oracle's own Philox implementation.
#include <rocrand/rocrand_philox4x32_10.h>

#include <cstdio>

struct Engine : rocrand_device::philox4x32_10_engine {
  uint4 rounds(uint4 c, uint2 k) { return ten_rounds(c, k); }
};

int main() {
  Engine e;
  unsigned c0, c1, c2, c3, k0, k1;
  while (std::scanf("%x %x %x %x %x %x", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
    uint4 r = e.rounds(uint4{c0, c1, c2, c3}, uint2{k0, k1});
    std::printf("%08x %08x %08x %08x\n", r.x, r.y, r.z, r.w);
  }
  return 0;
}
