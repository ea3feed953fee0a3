// Test-only pin: prints rocRAND's Philox4x32-10 block function for the
// (counter, key) pairs given on stdin, one "c0 c1 c2 c3 k0 k1" line each
// (hex).  rocRAND's engine is independent open-source code shipped with
// ROCm; the oracle's Philox is checked against it bit for bit.
#include <cstdio>
#include <rocrand/rocrand_philox4x32_10.h>

struct probe : rocrand_device::philox4x32_10_engine {
    uint4 block(uint4 c, uint2 k) { return ten_rounds(c, k); }
};

int main() {
    unsigned c0, c1, c2, c3, k0, k1;
    probe p;
    while (std::scanf("%x %x %x %x %x %x", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
        uint4 c; c.x = c0; c.y = c1; c.z = c2; c.w = c3;
        uint2 k; k.x = k0; k.y = k1;
        uint4 r = p.block(c, k);
        std::printf("%08x %08x %08x %08x\n", r.x, r.y, r.z, r.w);
    }
    return 0;
}
