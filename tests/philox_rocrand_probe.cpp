// Third-party cross-check for the oracle's Philox4x32-10: evaluates rocRAND's
// header implementation on the host for counters/keys read from stdin
// (one "c0 c1 c2 c3 k0 k1" line each, decimal) and prints the four outputs.
// Used only by tests/test_oracle_pins.py.
#include <cstdio>
#include <rocrand/rocrand_philox4x32_10.h>

struct Probe : rocrand_device::philox4x32_10_engine {
    uint4 eval(uint4 c, uint2 k) { return ten_rounds(c, k); }
};

int main() {
    Probe p;
    unsigned c0, c1, c2, c3, k0, k1;
    while (std::scanf("%u %u %u %u %u %u", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
        uint4 r = p.eval(uint4{c0, c1, c2, c3}, uint2{k0, k1});
        std::printf("%u %u %u %u\n", r.x, r.y, r.z, r.w);
    }
    return 0;
}
