// Test helper: prints Philox4x32-10 blocks computed by the rocRAND library's
// own engine, for a list of (counter, key) pairs read from stdin
// (six unsigned integers per line: c0 c1 c2 c3 k0 k1).  Used only to pin the
// oracle's independent Philox implementation against a published library.
#include <hip/hip_runtime.h>
#include <rocrand/rocrand_kernel.h>
#include <cstdio>

struct engine_probe : rocrand_device::philox4x32_10_engine {
    uint4 block(uint4 c, uint2 k) { return ten_rounds(c, k); }
};

int main()
{
    engine_probe p;
    unsigned c0, c1, c2, c3, k0, k1;
    while (std::scanf("%u %u %u %u %u %u", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
        uint4 r = p.block(uint4{c0, c1, c2, c3}, uint2{k0, k1});
        std::printf("%u %u %u %u\n", r.x, r.y, r.z, r.w);
    }
    return 0;
}
