// Test helper: evaluates rocRAND's Philox4x32-10 block function on the host for
// counters/keys read from stdin ("c0 c1 c2 c3 k0 k1" per line, decimal) and
// prints the four output words.  It runs the installed open-source rocRAND
// headers as an independent implementation to check the oracle against.
#include <cstdio>
#include <rocrand/rocrand_philox4x32_10.h>

struct block_probe : rocrand_device::philox4x32_10_engine {
    uint4 eval(uint4 c, uint2 k) { return ten_rounds(c, k); }
};

int main() {
    unsigned c0, c1, c2, c3, k0, k1;
    block_probe probe;
    while (std::scanf("%u %u %u %u %u %u", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
        uint4 c = {c0, c1, c2, c3};
        uint2 k = {k0, k1};
        uint4 r = probe.eval(c, k);
        std::printf("%u %u %u %u\n", r.x, r.y, r.z, r.w);
    }
    return 0;
}
