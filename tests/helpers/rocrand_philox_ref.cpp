// Independent Philox4x32-10 for pinning the oracle: evaluates rocRAND's own
// host-callable philox4x32_10 engine (its protected ten-round function) on
// counters read from stdin.  Input lines: "c0 c1 c2 c3 k0 k1" (decimal);
// output lines: the four 32-bit result words (decimal).
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>

struct Probe : rocrand_device::philox4x32_10_engine {
  uint4 eval(uint4 c, uint2 k) { return this->ten_rounds(c, k); }
};

int main() {
  Probe p;
  unsigned c0, c1, c2, c3, k0, k1;
  while (std::scanf("%u %u %u %u %u %u", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
    uint4 r = p.eval(make_uint4(c0, c1, c2, c3), make_uint2(k0, k1));
    std::printf("%u %u %u %u\n", r.x, r.y, r.z, r.w);
  }
  return 0;
}
