// Host-only program: Philox4x32-10 blocks from rocRAND's open-source engine,
// an implementation independent of the oracle's.  Reads "c0 c1 c2 c3 k0 k1"
// lines (decimal) on stdin and prints the four output words per line.
#include <hip/hip_runtime.h>
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>

struct Block : rocrand_device::philox4x32_10_engine {
    static uint4 of(uint4 c, uint2 k) { Block b; return b.ten_rounds(c, k); }
};

int main() {
    unsigned c0, c1, c2, c3, k0, k1;
    while (std::scanf("%u %u %u %u %u %u", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
        uint4 r = Block::of(uint4{c0, c1, c2, c3}, uint2{k0, k1});
        std::printf("%u %u %u %u\n", r.x, r.y, r.z, r.w);
    }
    return 0;
}
