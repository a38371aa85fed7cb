// Reads lines "c0 c1 c2 c3 k0 k1" (hex) and prints Philox4x32-10 of that
// counter and key as computed by rocRAND's engine (an implementation written
// and validated independently of this project).  Test helper only.
#include <rocrand/rocrand_philox4x32_10.h>

#include <cstdio>

int main()
{
    unsigned c0, c1, c2, c3, k0, k1;
    while (std::scanf("%x %x %x %x %x %x", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
        // The engine's counter holds (offset / 4) in words 0-1 and the
        // subsequence in words 2-3; its key is the 64-bit seed.  Offsets
        // count 32-bit outputs, so words 0-1 are advanced in four steps of
        // at most 2^62 counters each.
        unsigned long long seed = (static_cast<unsigned long long>(k1) << 32) | k0;
        unsigned long long sub = (static_cast<unsigned long long>(c3) << 32) | c2;
        unsigned long long lo = (static_cast<unsigned long long>(c1) << 32) | c0;
        rocrand_device::philox4x32_10_engine e(seed, sub, 0);
        for (int i = 0; i < 4; ++i) e.discard((lo / 4) * 4);
        e.discard((lo % 4) * 4);
        uint4 r = e.next4();
        std::printf("%08x %08x %08x %08x\n", r.x, r.y, r.z, r.w);
    }
    return 0;
}
