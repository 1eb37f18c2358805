// Prints rocRAND's Philox4x32-10 block function for (counter, key) pairs read
// from stdin ("c0 c1 c2 c3 k0 k1" per line, decimal).  Used by the CPU tests
// as an implementation independent of the oracle's own Philox.
#include <cstdio>
#include <rocrand/rocrand_philox4x32_10.h>

struct Probe : rocrand_device::philox4x32_10_engine {
    static uint4 block(uint4 c, uint2 k) { Probe p; return p.ten_rounds(c, k); }
};

int main() {
    unsigned c0, c1, c2, c3, k0, k1;
    while (std::scanf("%u %u %u %u %u %u", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
        uint4 r = Probe::block(uint4{c0, c1, c2, c3}, uint2{k0, k1});
        std::printf("%u %u %u %u\n", r.x, r.y, r.z, r.w);
    }
    return 0;
}
