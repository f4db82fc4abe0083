// Prints rocRAND's Philox4x32-10 block function for counters/keys read from
// stdin ("c0 c1 c2 c3 k0 k1" per line, hex).  Used only to cross-check the
// oracle's generator against an independent published implementation.
#include <cstdio>
#include <rocrand/rocrand_philox4x32_10.h>

struct Expose : rocrand_device::philox4x32_10_engine {
    uint4 block(uint4 c, uint2 k) { return ten_rounds(c, k); }
};

int main()
{
    unsigned c0, c1, c2, c3, k0, k1;
    Expose e;
    while (std::scanf("%x %x %x %x %x %x", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
        uint4 c = {c0, c1, c2, c3};
        uint2 k = {k0, k1};
        uint4 r = e.block(c, k);
        std::printf("%08x %08x %08x %08x\n", r.x, r.y, r.z, r.w);
    }
    return 0;
}
