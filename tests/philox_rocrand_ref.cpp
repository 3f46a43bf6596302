// Host-side reference for Philox4x32-10 taken from rocRAND's own engine
// (an independent implementation), used only to pin the oracle's generator.
// Reads "c0 c1 c2 c3 k0 k1" (hex) per line, prints the four output words.
#include <hip/hip_runtime.h>
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>

struct Engine : rocrand_device::philox4x32_10_engine {
    uint4 rounds(uint4 c, uint2 k) { return this->ten_rounds(c, k); }
};

int main()
{
    Engine e;
    unsigned v[6];
    while (std::scanf("%x %x %x %x %x %x", &v[0], &v[1], &v[2], &v[3], &v[4], &v[5]) == 6) {
        uint4 r = e.rounds(uint4{v[0], v[1], v[2], v[3]}, uint2{v[4], v[5]});
        std::printf("%08x %08x %08x %08x\n", r.x, r.y, r.z, r.w);
    }
    return 0;
}
