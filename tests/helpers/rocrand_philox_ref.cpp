// Independent Philox4x32-10 reference for the tests: rocRAND's engine (a
// library implementation from its published definition), driven on the host.
// Reads n records of (c0 c1 c2 c3 k0 k1) as little-endian u32 from stdin and
// writes n x 4 u32 outputs to stdout.
#include <rocrand/rocrand_philox4x32_10.h>

#include <cstdint>
#include <cstdio>
#include <vector>

struct Reference : rocrand_device::philox4x32_10_engine {
    uint4 block(uint4 c, uint2 k) { return ten_rounds(c, k); }
};

int main() {
    Reference ref;
    std::vector<uint32_t> rec(6);
    while (std::fread(rec.data(), 4, 6, stdin) == 6) {
        uint4 c = {rec[0], rec[1], rec[2], rec[3]};
        uint2 k = {rec[4], rec[5]};
        uint4 r = ref.block(c, k);
        uint32_t o[4] = {r.x, r.y, r.z, r.w};
        std::fwrite(o, 4, 4, stdout);
    }
    return 0;
}
