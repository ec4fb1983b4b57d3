// Reference Philox4x32-10 block function from rocRAND (library routine), used by
// the CPU pin test of the oracle generator.  Reads "c0 c1 c2 c3 k0 k1" (hex) per line.
#include <hip/hip_runtime.h>
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>
struct raw_philox : rocrand_device::philox4x32_10_engine {
  uint4 block(uint4 c, uint2 k) { return ten_rounds(c, k); }
};
int main() {
  unsigned c[4], k[2];
  raw_philox e;
  while (scanf("%x %x %x %x %x %x", &c[0], &c[1], &c[2], &c[3], &k[0], &k[1]) == 6) {
    uint4 r = e.block(uint4{c[0], c[1], c[2], c[3]}, uint2{k[0], k[1]});
    printf("%08x %08x %08x %08x\n", r.x, r.y, r.z, r.w);
  }
  return 0;
}
