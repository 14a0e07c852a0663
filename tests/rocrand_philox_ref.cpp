// Host-side reference values of Philox4x32-10 taken from rocRAND's engine
// (an implementation independent of this repository), used to pin the
// oracle's own Philox.  Reads lines "c0 c1 c2 c3 k0 k1" (hex) from stdin and
// prints the four output words of the ten-round bijection for each.
#include <cstdio>
#include <rocrand/rocrand_philox4x32_10.h>

// rocRAND keeps the raw counter->output map protected; expose it.
struct raw_philox : rocrand_device::philox4x32_10_engine {
    using rocrand_device::philox4x32_10_engine::ten_rounds;
};

int main() {
    unsigned c[4], k[2];
    raw_philox eng;
    while (std::scanf("%x %x %x %x %x %x", &c[0], &c[1], &c[2], &c[3], &k[0], &k[1]) == 6) {
        uint4 ctr = {c[0], c[1], c[2], c[3]};
        uint2 key = {k[0], k[1]};
        uint4 o = eng.ten_rounds(ctr, key);
        std::printf("%08x %08x %08x %08x\n", o.x, o.y, o.z, o.w);
    }
    return 0;
}
