// Independent Philox4x32-10 reference for the oracle's generator pin.
//
// Reads lines "c0 c1 c2 c3 k0 k1" on stdin and prints the four output words
// of ten Philox4x32 rounds, as computed by rocRAND's open-source header
// implementation of the generator of Salmon et al. (SC'11).  Built for the
// host only; it never touches a GPU.
#include <hip/hip_runtime.h>
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>

struct Rounds : rocrand_device::philox4x32_10_engine {
    uint4 run(uint4 c, uint2 k) { return ten_rounds(c, k); }
};

int main()
{
    Rounds e;
    unsigned a, b, c, d, k0, k1;
    while (std::scanf("%u %u %u %u %u %u", &a, &b, &c, &d, &k0, &k1) == 6) {
        uint4 r = e.run(uint4{a, b, c, d}, uint2{k0, k1});
        std::printf("%u %u %u %u\n", r.x, r.y, r.z, r.w);
    }
    return 0;
}
