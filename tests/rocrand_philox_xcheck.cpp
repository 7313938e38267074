#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>
struct Exposed : rocrand_device::philox4x32_10_engine {
  uint4 block(uint4 c, uint2 k) { return ten_rounds(c, k); }
};
int main() {
  unsigned c0,c1,c2,c3,k0,k1;
  Exposed e;
  while (scanf("%x %x %x %x %x %x", &c0,&c1,&c2,&c3,&k0,&k1) == 6) {
    uint4 r = e.block(uint4{c0,c1,c2,c3}, uint2{k0,k1});
    printf("%08x %08x %08x %08x\n", r.x, r.y, r.z, r.w);
  }
}
