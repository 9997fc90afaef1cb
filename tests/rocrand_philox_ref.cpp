// Reference Philox4x32-10 outputs from rocRAND's host-callable engine (a
// third-party implementation), used to pin the oracle's own Philox.
// Reads lines "c0 c1 c2 c3 k0 k1" on stdin, prints the four output words.
#include <hip/hip_runtime.h>
#include <rocrand/rocrand_kernel.h>

#include <cstdio>

namespace {
// the ten-round block function is a protected member of the engine
struct Block : rocrand_device::philox4x32_10_engine {
    uint4 apply(uint4 ctr, uint2 key) { return ten_rounds(ctr, key); }
};
}  // namespace

int main()
{
    Block engine;
    unsigned c0, c1, c2, c3, k0, k1;
    while (std::scanf("%u %u %u %u %u %u", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
        uint4 out = engine.apply(uint4{c0, c1, c2, c3}, uint2{k0, k1});
        std::printf("%u %u %u %u\n", out.x, out.y, out.z, out.w);
    }
    return 0;
}
