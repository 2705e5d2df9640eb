// Host-side Philox4x32-10 from rocRAND's open-source header, used only as an
// independent implementation that the oracle's generator is checked against.
// Reads lines "c0 c1 c2 c3 k0 k1" and prints the four output words.
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>

struct Engine : rocrand_device::philox4x32_10_engine {
  uint4 run(uint4 c, uint2 k) { return ten_rounds(c, k); }
};

int main() {
  Engine e;
  unsigned a[6];
  while (std::scanf("%u %u %u %u %u %u", a, a + 1, a + 2, a + 3, a + 4, a + 5) == 6) {
    uint4 c = {a[0], a[1], a[2], a[3]};
    uint2 k = {a[4], a[5]};
    uint4 r = e.run(c, k);
    std::printf("%u %u %u %u\n", r.x, r.y, r.z, r.w);
  }
  return 0;
}
