// Prints rocRAND's Philox4x32-10 block outputs for counters/keys read from
// stdin (hex words: c0 c1 c2 c3 k0 k1 per line).  rocRAND is an independent
// implementation of the same published generator; the oracle's Philox is
// checked against it.  Host code only.
#include <cstdio>
#include <rocrand/rocrand_philox4x32_10.h>

// The block function is a protected member; a derived class exposes it.
struct philox_block : rocrand_device::philox4x32_10_engine
{
    using rocrand_device::philox4x32_10_engine::ten_rounds;
};

int main()
{
    unsigned c0, c1, c2, c3, k0, k1;
    philox_block eng;
    while (std::scanf("%x %x %x %x %x %x", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
        uint4 ctr{c0, c1, c2, c3};
        uint2 key{k0, k1};
        uint4 out = eng.ten_rounds(ctr, key);
        std::printf("%08x %08x %08x %08x\n", out.x, out.y, out.z, out.w);
    }
    return 0;
}
