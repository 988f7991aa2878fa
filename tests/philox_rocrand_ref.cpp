// Independent reference for Philox4x32-10 used only by the CPU test suite:
// ROCm's open-source rocRAND device/host implementation of the same published
// generator (Salmon et al., SC'11).  Reads "c0 c1 c2 c3 k0 k1" per line on
// stdin and prints the four output words in hex.  Host code only.
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>

struct Engine : rocrand_device::philox4x32_10_engine {
    using philox4x32_10_engine::ten_rounds;
};

int main()
{
    Engine e;
    unsigned c0, c1, c2, c3, k0, k1;
    while (std::scanf("%u %u %u %u %u %u", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
        uint4 o = e.ten_rounds(uint4{c0, c1, c2, c3}, uint2{k0, k1});
        std::printf("%08x %08x %08x %08x\n", o.x, o.y, o.z, o.w);
    }
    return 0;
}
